// Storage pool of the H-LU factors: host bookkeeping over memory chunks
// that the chunk type provides (device buffers in the library).  The chunk
// type has members p (element pointer) and n (element count), alloc(count),
// and is movable.
#pragma once
#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>
#include <set>
#include <utility>
#include <vector>

namespace cbie {

// Buffers (multiples of 32 elements) are carved best-fit from the chunks;
// a freed range is merged with the free neighbours of its chunk, so that the
// memory of factors whose rank changed serves factors of any other size.  A
// released buffer may still be read or written by tasks recorded before its
// release, so it is reused only after the stream has completed them:
// released while a program is being recorded -> waiting for that program's
// launch (tagged with its launch number) -> free once the stream has
// completed that program (completed_through) or has been synchronized
// (completed).
template <typename E, typename Chunk> struct FactorPool {
    using P = E*;
    struct Range {
        size_t n;
        int chunk;
    };
    std::vector<Chunk> chunks;
    std::map<P, int> chunk_at;                    // chunk base -> index
    std::map<P, Range> free_at;                   // free ranges by address
    std::set<std::pair<size_t, P>> free_by_size;  // the same, by size
    struct Pending {
        P p;
        size_t n;
        int64_t gen;   // launch number of the program it waits for
    };
    std::vector<std::pair<P, size_t>> rec;
    std::vector<Pending> run;
    int64_t launches = 0;   // programs launched so far (the next one gets this number)
    size_t chunk_elems = size_t(1) << 26;
    size_t live = 0, peak = 0;
    static size_t rounded(size_t n) { return std::max<size_t>(32, (n + 31) & ~size_t(31)); }
    void add_free(P p, size_t n, int chunk) {
        auto nx = free_at.find(p + n);
        if (nx != free_at.end() && nx->second.chunk == chunk) {
            free_by_size.erase({nx->second.n, nx->first});
            n += nx->second.n;
            free_at.erase(nx);
        }
        auto it = free_at.lower_bound(p);
        if (it != free_at.begin()) {
            auto pv = std::prev(it);
            if (pv->second.chunk == chunk && pv->first + pv->second.n == p) {
                free_by_size.erase({pv->second.n, pv->first});
                p = pv->first;
                n += pv->second.n;
                free_at.erase(pv);
            }
        }
        free_at[p] = Range{n, chunk};
        free_by_size.insert({n, p});
    }
    P alloc(size_t n) {
        n = rounded(n);
        auto it = free_by_size.lower_bound({n, nullptr});
        if (it == free_by_size.end()) {
            Chunk b;
            b.alloc(std::max(n, chunk_elems));
            const int id = (int)chunks.size();
            chunks.push_back(std::move(b));
            chunk_at[chunks.back().p] = id;
            add_free(chunks.back().p, chunks.back().n, id);
            it = free_by_size.lower_bound({n, nullptr});
        }
        const size_t have = it->first;
        const P p = it->second;
        free_by_size.erase(it);
        auto fr = free_at.find(p);
        const int chunk = fr->second.chunk;
        free_at.erase(fr);
        if (have > n) {
            free_at[p + n] = Range{have - n, chunk};
            free_by_size.insert({have - n, p + n});
        }
        live += n;
        peak = std::max(peak, live);
        return p;
    }
    // n: the size passed to alloc
    void release(P p, size_t n) {
        if (!p) return;
        n = rounded(n);
        rec.push_back({p, n});
        live -= n;
    }
    void launched() {
        for (const auto& x : rec) run.push_back(Pending{x.first, x.second, launches});
        rec.clear();
        ++launches;
    }
    // every program with launch number <= g has completed on the stream
    void completed_through(int64_t g) {
        size_t keep = 0;
        for (size_t i = 0; i < run.size(); ++i) {
            if (run[i].gen <= g) {
                auto c = std::prev(chunk_at.upper_bound(run[i].p));
                add_free(run[i].p, run[i].n, c->second);
            } else {
                run[keep++] = run[i];
            }
        }
        run.resize(keep);
    }
    void completed() { completed_through(launches - 1); }
    double capacity() const {
        double c = 0;
        for (const auto& b : chunks) c += (double)b.n;
        return c;
    }
};

}  // namespace cbie
