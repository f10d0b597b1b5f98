// Autotuner: picks the launch shape of a factor-and-solve by timing it on
// the device -- the chain length of the finest level (block_rows), the lane
// mapping of its factor kernel (segment width or rows) and the chain length
// of the reduced levels (coarse_rows) -- and caches the choice per shape
// class of the system.  The method computes the same solution (up to
// rounding) for every choice; only the time differs.
#include "pf.h"
#include "pf_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

using namespace pf;

namespace {

int padded(int m)
{
    int M = 1;
    while (M < m) M <<= 1;
    return M;
}

// shape class: kind, padded block size, precision, size bucket (half
// octaves of nb), right-hand sides (1, 2-4, 5-16, more)
using Key = std::tuple<int, int, int, int, int>;

Key key_of(const pf_matrix *A, const pf_opts &o, int nrhs)
{
    const int sb = (int)std::lround(2.0 * std::log2((double)std::max<int64_t>(A->nb, 2)));
    const int rb = nrhs <= 1 ? 1 : nrhs <= 4 ? 4 : nrhs <= 16 ? 16 : 64;
    return Key{A->kind, padded(A->m), o.prec, sb, rb};
}

struct Entry {
    pf_opts opts;
    float ms;
};

std::mutex g_mu;
std::map<Key, Entry> g_cache;

// median of a few timed factor-and-solve calls; < 0 on failure
float time_candidate(const pf_matrix *A, const pf_opts &o, int nrhs, const double *f, double *x,
                     hipStream_t s)
{
    pf_factor_t F = nullptr;
    if (pf_factor(A, &o, s, &F) != 0) return -1.f;
    const int64_t n = A->nb * A->m;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best = -1.f;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        std::vector<float> t;
        bool ok = pf_factor_solve(F, nrhs, f, n, x, n, s, nullptr) == 0;   // warm-up
        for (int rep = 0; ok && rep < 3; ++rep) {
            ok = hipEventRecord(e0, s) == hipSuccess &&
                 pf_factor_solve(F, nrhs, f, n, x, n, s, nullptr) == 0 &&
                 hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.f;
            if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) t.push_back(ms);
        }
        if (ok && !t.empty()) {
            std::sort(t.begin(), t.end());
            best = t[t.size() / 2];
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    pf_destroy(F);
    return best;
}

}  // namespace

extern "C" int pf_autotune(const pf_matrix *A, const pf_opts *base, int32_t nrhs, void *stream,
                           pf_opts *best, float *best_ms)
{
    if (!A) return -1;
    if (nrhs < 1) return -3;
    if (!best) return -5;
    pf_opts o0{};
    if (base) o0 = *base;
    o0.flags &= ~PF_FLAG_AUTOTUNE;
    o0.partitions = 0;
    o0.block_rows = o0.coarse_rows = o0.lane_entries = 0;
    if (pf_factor_bytes(A, &o0) == 0) return -1;   // the checks pf_factor applies
    hipStream_t s = (hipStream_t)stream;
    const int M = padded(A->m);
    const int64_t n = A->nb * A->m;
    double *f = nullptr, *x = nullptr;
    if (hipMallocAsync((void **)&f, (size_t)n * nrhs * sizeof(double), s) != hipSuccess)
        return PF_ENOMEM;
    if (hipMallocAsync((void **)&x, (size_t)n * nrhs * sizeof(double), s) != hipSuccess) {
        hipFreeAsync(f, s);
        return PF_ENOMEM;
    }
    if (launch_fill_u64((unsigned long long *)f, n * nrhs, 0x3FF0000000000000ull, s) != hipSuccess) {   // f = 1
        hipFreeAsync(f, s);
        hipFreeAsync(x, s);
        return PF_EHIP;
    }

    // candidate mappings of the finest level: the segment widths with a
    // kernel for this block size, and rows
    std::vector<std::pair<int, int>> maps;   // (lane_entries, flags)
    for (int E = 1; E <= M; E <<= 1)
        if (seg_ok(M, E)) maps.push_back({E, 0});
    maps.push_back({0, PF_FLAG_MAP_ROWS});
    const int rows0[] = {4, 8, 12, 16, 24, 32};
    const int rowsc[] = {2, 3, 4, 6};

    pf_opts bo = o0;
    float bms = -1.f;
    auto consider = [&](const pf_opts &o) {
        const float ms = time_candidate(A, o, nrhs, f, x, s);
        if (ms > 0.f && (bms < 0.f || ms < bms)) {
            bms = ms;
            bo = o;
        }
    };
    consider(o0);   // the planner's own choice
    for (const auto &mp : maps)
        for (int L : rows0) {
            if (L > A->nb / 2) continue;
            pf_opts o = o0;
            o.lane_entries = mp.first;
            o.flags |= mp.second;
            o.block_rows = L;
            o.coarse_rows = 3;
            consider(o);
        }
    const pf_opts level0 = bo;
    for (int L : rowsc) {
        if (L == 3) continue;
        pf_opts o = level0;
        o.coarse_rows = L;
        consider(o);
    }
    hipFreeAsync(f, s);
    hipFreeAsync(x, s);
    hipStreamSynchronize(s);
    if (bms < 0.f) return PF_EHIP;
    *best = bo;
    if (best_ms) *best_ms = bms;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key_of(A, o0, nrhs)] = Entry{bo, bms};
    return 0;
}

extern "C" void pf_autotune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
}

namespace pf {

// The options a PF_FLAG_AUTOTUNE factorization uses: the cached choice for
// the system's shape class, tuned now (on this matrix) if there is none.
int tuned_opts(const pf_matrix *A, const pf_opts &o, int nrhs, hipStream_t s, pf_opts *out)
{
    pf_opts base = o;
    base.flags &= ~PF_FLAG_AUTOTUNE;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key_of(A, base, nrhs));
        if (it != g_cache.end()) {
            *out = it->second.opts;
            out->prec = base.prec;
            out->max_refine = base.max_refine;
            out->tol = base.tol;
            out->flags = (out->flags & PF_FLAG_MAP_ROWS) | (base.flags & ~PF_FLAG_MAP_ROWS);
            return 0;
        }
    }
    pf_opts best{};
    const int rc = pf_autotune(A, &base, nrhs, s, &best, nullptr);
    if (rc) return rc;
    *out = best;
    out->flags = (best.flags & PF_FLAG_MAP_ROWS) | (base.flags & ~PF_FLAG_MAP_ROWS);
    return 0;
}

}  // namespace pf
