// Stages not yet implemented in this build step.
#include "ctx.hpp"

namespace cbie {
struct HMat {};
Ctx::Ctx() {}
Ctx::~Ctx() {}
void stage_factor(Ctx&, int) { throw Error{CBIE_EINTERNAL, "factor: not implemented"}; }
void stage_solve(Ctx&, int, const zd*, zd*, long, double, int, int*) { throw Error{CBIE_EINTERNAL, "solve: not implemented"}; }
}  // namespace cbie
