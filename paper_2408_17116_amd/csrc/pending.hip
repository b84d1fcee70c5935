// Stages not yet implemented in this build step.
#include "ctx.hpp"

namespace cbie {
struct HMat {};
Ctx::Ctx() {}
Ctx::~Ctx() {}
void stage_compress(Ctx&, double, int) { throw Error{CBIE_EINTERNAL, "compress: not implemented"}; }
void stage_factor(Ctx&, int) { throw Error{CBIE_EINTERNAL, "factor: not implemented"}; }
void stage_solve(Ctx&, int, const zd*, zd*, long, double, int, int*) { throw Error{CBIE_EINTERNAL, "solve: not implemented"}; }
void stage_matvec(Ctx&, int, const zd*, zd*, long) { throw Error{CBIE_EINTERNAL, "matvec: not implemented"}; }
void stage_rhs(Ctx&, int, const double*, const double*, zd*, long) { throw Error{CBIE_EINTERNAL, "rhs: not implemented"}; }
void stage_farfield(Ctx&, int, const zd*, long, int, const double*, zd*) { throw Error{CBIE_EINTERNAL, "farfield: not implemented"}; }
void export_lowrank(Ctx&, zd*, long) { throw Error{CBIE_EINTERNAL, "export: not implemented"}; }
}  // namespace cbie
