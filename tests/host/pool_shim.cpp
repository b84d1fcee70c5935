// Test shim: the library's factor-storage pool over host memory chunks,
// driven by seeded sequences of allocations and deferred releases, with its
// invariants checked after every step.  Built with the host compiler by the
// CPU tests.
#include <cstdint>
#include <cstdlib>
#include <random>
#include <vector>

#include "pool.hpp"

namespace {
struct HostChunk {
    double* p = nullptr;
    size_t n = 0;
    HostChunk() = default;
    HostChunk(HostChunk&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    HostChunk& operator=(HostChunk&& o) noexcept { std::swap(p, o.p); std::swap(n, o.n); return *this; }
    ~HostChunk() { free(p); }
    void alloc(size_t c) { free(p); p = static_cast<double*>(malloc(c * sizeof(double))); n = c; }
};
using Pool = cbie::FactorPool<double, HostChunk>;

struct Live {
    double* p;
    size_t n;      // requested size
    uint32_t tag;  // written over the whole buffer
};

// 0 = fine; otherwise the number of the violated check
int check(const Pool& P, const std::vector<Live>& live, std::vector<std::pair<double*, size_t>>& iv) {
    iv.clear();
    size_t lsum = 0, fsum = 0, pend = 0;
    for (const Live& a : live) {
        iv.push_back({a.p, Pool::rounded(a.n)});
        lsum += Pool::rounded(a.n);
        // every live buffer lies inside one chunk
        auto c = std::prev(P.chunk_at.upper_bound(a.p));
        const auto& ch = P.chunks[c->second];
        if (a.p < ch.p || a.p + Pool::rounded(a.n) > ch.p + ch.n) return 1;
        // and still holds what was written into it
        for (size_t e = 0; e < a.n; e += 7)
            if (a.p[e] != (double)a.tag) return 2;
    }
    for (const auto& f : P.free_at) {
        iv.push_back({f.first, f.second.n});
        fsum += f.second.n;
        // a free range never touches a free neighbour of its chunk
        auto nx = P.free_at.find(f.first + f.second.n);
        if (nx != P.free_at.end() && nx->second.chunk == f.second.chunk) return 3;
    }
    for (const auto& x : P.rec) { iv.push_back(x); pend += x.second; }
    for (const auto& x : P.run) {
        iv.push_back({x.p, x.n});
        pend += x.n;
        if (x.gen < 0 || x.gen >= P.launches) return 8;   // waits for a program that was launched
    }
    std::sort(iv.begin(), iv.end());
    for (size_t k = 1; k < iv.size(); ++k)
        if (iv[k].first < iv[k - 1].first + iv[k - 1].second) return 4;   // overlap
    if ((double)(lsum + fsum + pend) != P.capacity()) return 5;           // every element accounted for
    if (P.free_at.size() != P.free_by_size.size()) return 6;
    if (P.live != lsum || P.peak < P.live) return 7;
    return 0;
}
}  // namespace

// Random allocations (sizes up to max_elems) and releases, with program
// launches and completions in between.  out: [capacity, peak].
extern "C" int pool_random(unsigned seed, int steps, size_t chunk_elems, size_t max_elems, double* out) {
    Pool P;
    P.chunk_elems = chunk_elems;
    std::mt19937 g(seed);
    std::vector<Live> live;
    std::vector<std::pair<double*, size_t>> iv;
    for (int it = 0; it < steps; ++it) {
        const int op = (int)(g() % 8);
        if (op < 4 || live.empty()) {
            Live a;
            a.n = 1 + g() % max_elems;
            a.p = P.alloc(a.n);
            a.tag = g();
            for (size_t e = 0; e < a.n; ++e) a.p[e] = (double)a.tag;
            live.push_back(a);
        } else if (op < 7) {
            const size_t i = g() % live.size();
            P.release(live[i].p, live[i].n);
            live.erase(live.begin() + i);
        } else {
            // a launch; then the stream has passed every program, or all but
            // the last one (an event after the previous program), or none
            P.launched();
            const int r = (int)(g() % 3);
            if (r == 1) P.completed();
            if (r == 2) {
                P.completed_through(P.launches - 2);
                for (const auto& x : P.run)
                    if (x.gen != P.launches - 1) return 9;   // only the last program's releases remain
            }
        }
        if (const int e = check(P, live, iv)) return 100 * e + 0 * it;
    }
    for (const Live& a : live) P.release(a.p, a.n);
    P.launched();
    P.completed();
    // everything free again: one merged range per chunk
    if (P.free_at.size() != P.chunks.size()) return 900;
    out[0] = P.capacity();
    out[1] = (double)P.peak;
    return 0;
}

// Low-rank factors whose ranks grow: n_blocks buffers of m x r elements, each
// round every block's buffer replaced by one of rank r + dr (released after
// the round's program, as in the factorization).  out: [capacity, peak,
// largest live + pending storage, the least any pool could hold].
extern "C" int pool_growing_ranks(int n_blocks, int m, int r0, int dr, int rounds, size_t chunk_elems, double* out) {
    Pool P;
    P.chunk_elems = chunk_elems;
    std::vector<Live> live(n_blocks);
    std::vector<std::pair<double*, size_t>> iv;
    double need = 0.0;
    for (int b = 0; b < n_blocks; ++b) {
        live[b] = Live{P.alloc((size_t)m * r0), (size_t)m * r0, (uint32_t)b};
        for (size_t e = 0; e < live[b].n; ++e) live[b].p[e] = (double)b;
    }
    for (int k = 1; k <= rounds; ++k) {
        for (int b = 0; b < n_blocks; ++b) {
            const size_t n = (size_t)m * (r0 + k * dr);
            double* q = P.alloc(n);
            for (size_t e = 0; e < n; ++e) q[e] = (double)b;
            P.release(live[b].p, live[b].n);
            live[b].p = q;
            live[b].n = n;
        }
        size_t pend = 0;
        for (const auto& x : P.rec) pend += x.second;
        need = std::max(need, (double)(P.live + pend));
        P.launched();
        P.completed();
        if (const int e = check(P, live, iv)) return 100 * e;
    }
    out[0] = P.capacity();
    out[1] = (double)P.peak;
    out[2] = need;
    return 0;
}
