// Host side of the partition-method library: argument checks, the level
// plan of the recursion, device memory of a factor handle, the solve
// orchestration (forward sweeps down the levels, back substitution up) and
// FP64 iterative refinement.
#include "pf.h"
#include "pf_internal.h"
#include "kernels_tri.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <tuple>
#include <vector>

using namespace pf;

namespace {

// PF_FLAG_ENLARGE: room for the codes of failing partitions per pass
constexpr int kBadCap = 16384;

struct Level {
    int kind = PF_BTRI;
    int64_t nb = 0, p = 1;
    bool f32 = false;
    int seg = 0;          // factor lane mapping: E entries per lane (segments), 0 = rows,
                          // kMapMfma / kMapMfma32 = matrix-core products (m = 8 finest
                          // level / m = 32)
    const double *D = nullptr, *Dadd = nullptr, *Lo = nullptr, *Up = nullptr, *C = nullptr;
    void *E = nullptr, *R = nullptr, *Z = nullptr, *X = nullptr;
    double *nD = nullptr, *nDadd = nullptr, *nLo = nullptr, *nUp = nullptr, *nC = nullptr;
    std::vector<int64_t> seps;   // explicit partition boundaries (empty: balanced)
    int64_t *d_sep = nullptr;    // their device copy
};

struct PlanLevel {
    int kind;
    int64_t nb, p;
    std::vector<int64_t> seps;   // explicit partition boundaries, p + 1 (empty: balanced)
};

// Explicit partition boundaries per level (enlarged reduced systems).
using SepOverrides = std::map<int, std::vector<int64_t>>;

// One device allocation carved into the memory of many handles (a batch).
// Shared by the batch and by the handles it hands out; freed by the last.
// Device memory of handles and batches: the caller's allocator when one is
// set (pf_set_allocator), else stream-ordered hipMallocAsync / hipFreeAsync.
// Each handle and arena keeps the allocator it was created with, so that a
// later pf_set_allocator does not pair a block with the wrong free.
Allocator g_allocator;

// the most recent failing HIP call of this thread (pf_last_hip_error)
thread_local int g_last_hip = 0;

// PF_ENOMEM for an allocation that ran out of memory, PF_EHIP (and the code
// kept for pf_last_hip_error) for any other failure
int alloc_status(hipError_t e)
{
    g_last_hip = (int)e;
    return e == hipErrorOutOfMemory ? PF_ENOMEM : PF_EHIP;
}

hipError_t dev_alloc(const Allocator &a, void **p, size_t bytes, hipStream_t s)
{
    *p = nullptr;
    if (a.alloc) {
        *p = a.alloc(bytes, (void *)s, a.ctx);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMallocAsync(p, bytes, s);
}

void dev_free(const Allocator &a, void *p, size_t bytes, hipStream_t s)
{
    if (!p) return;
    if (a.free) a.free(p, bytes, (void *)s, a.ctx);
    else hipFreeAsync(p, s);
}

struct DevBlock {
    void *p;
    size_t bytes;
};

struct Arena {
    char *base = nullptr;
    size_t off = 0, cap = 0;
    bool counting = false;
    Allocator al;   // what base came from (dev_alloc)
    int refs = 0;
};

void arena_release(Arena *ar, hipStream_t s)
{
    if (--ar->refs > 0) return;
    dev_free(ar->al, ar->base, ar->cap, s);
    delete ar;
}

}  // namespace

struct pf_factor_s {
    pf_matrix A{};
    pf_opts opts{};
    int m = 0, M = 0;
    int64_t nb = 0;
    hipStream_t stream = nullptr;
    std::vector<Level> lv;
    Allocator al;                          // the allocator of its own blocks
    std::vector<DevBlock> allocs;
    unsigned long long *d_status = nullptr;
    unsigned long long *d_norm = nullptr;  // ||A||_inf bits
    void *d_dump = nullptr;                // target of masked stores (kDumpBytes)
    const double *d_zero = nullptr;        // kZeroBytes of zeros after the dump area
    // solve workspace
    int rhs_cap = 0;
    std::vector<double *> wsF, wsFadd, wsY;
    double *wsPadF = nullptr, *wsPadX = nullptr, *wsR = nullptr, *wsD = nullptr;
    unsigned long long *d_norms = nullptr;
    std::vector<DevBlock> ws_allocs;
    // optional per-launch timing
    struct ProfSlot {
        int phase = 0, level = 0;
        hipEvent_t a = nullptr, b = nullptr;
    };
    bool prof = false;
    std::vector<ProfSlot> prof_fac, prof_sol;
    size_t prof_fac_n = 0, prof_sol_n = 0;
    // level-0 matrix padded to the instantiated block size (when M != m)
    double *padD = nullptr, *padLo = nullptr, *padUp = nullptr, *padC = nullptr;
    // set when the handle's memory is a slice of a batch's arena
    Arena *arena = nullptr;
    // PF_FLAG_ENLARGE: failing partitions' codes (kBadCap) and their count
    unsigned long long *d_badlist = nullptr;
    // small scalar tridiagonal systems: pf_factor_solve with one right-hand
    // side runs as one launch (local cyclic reduction, kernels_tri_cr.hip),
    // which leaves the stored factors behind the matrix's values
    bool tri_cr = false;
    bool factors_stale = false;
};

namespace {

int padded_block(int m)
{
    int M = 1;
    while (M < m) M <<= 1;
    return M;
}

// Blocks per partition (the chain length of one group of lanes).  Short
// chains give many partitions (parallelism, latency hiding); the reduced
// system then has about nb/(L+1) blocks and is solved by the next level.
int target_rows(int kind, int M, bool f32, int level, const pf_opts &o)
{
    if (level == 0 && o.block_rows > 0) return o.block_rows;
    if (level > 0 && o.coarse_rows > 0) return o.coarse_rows;
    // measured on MI355X for the m = 8 BVP (segment mapping, two entries per
    // lane at level 0): 16 blocks at level 0, where 3855 partitions fill the
    // resident wave slots about once, and 3 on the reduced levels (latency-
    // bound: the chain length per level trades against the number of levels).
    // The m = 16 bidiagonal-plus-corner form in FP64 (its matrix-core kernel
    // inverts four blocks at a time): 16 at level 0, which costs about as much
    // as 4 there and leaves a reduced system a quarter the size (m = 16 BVP,
    // N = 2^18: 0.97 vs 1.08 ms per step).
    if (level == 0) return (M <= 8 || (kind == PF_BABD && M == 16 && !f32)) ? 16 : 4;
    // scalar tridiagonal reduced levels run their chains out of LDS, where a
    // block row costs little: 8 blocks per partition (8 levels instead of 11
    // for n = 2^24, 0.696 vs 0.720 ms per step; n = 4096: 52 vs 59 us)
    if (kind == PF_BTRI && M == 1) return 8;
    return 3;
}

// The finest level's chains grow past the table where the level has
// partitions to spare: doubled, up to kSpareMaxChain blocks, while at least
// kSpareMinParts partitions remain (sixteen per SIMD of the GPU).  Longer
// chains cost the finest level little and shrink every reduced level (one
// system of 2^20 blocks, factor and solve: 32.2 -> 29.8 ms for m = 32 and
// 5.87 -> 5.14 ms for m = 16 with the rule's 32 blocks instead of 4; 1.35 ->
// 1.32 ms for m = 8 with 32 instead of 16; the bidiagonal-plus-corner form,
// m = 16, 2^18 blocks, FP32 factors and refinement: 3.17 -> 3.03 ms with 8
// instead of 4).  Batches apply the
// same rule to the rows of each grouped launch (batch_chain_lengths).
// Scalar systems keep the table: their LDS-staged kernels bound the chain.
constexpr int kSpareMaxChain = 64;
constexpr int64_t kSpareMinParts = 16384;
int spare_chain(int L, int64_t rows)
{
    while (2 * L <= kSpareMaxChain && rows / (2 * L + 1) >= kSpareMinParts) L *= 2;
    return L;
}
int finest_chain(int kind, int M, bool f32, int64_t nb, const pf_opts &o)
{
    const int L = target_rows(kind, M, f32, 0, o);
    return (o.block_rows > 0 || M == 1) ? L : spare_chain(L, nb);
}

constexpr int64_t kTail = 6;   // block tridiagonal systems this small: one chain

// Scalar tridiagonal systems of at most kTriCrMaxRows rows in FP64 are
// solved by pf_factor_solve (one right-hand side) in one launch with local
// cyclic reduction; by default their finest level then has partitions of
// about kTriCrRows rows (fewer reduction rounds), at most one wave's lanes of
// them (the reduced system is solved across one wave).
constexpr int64_t kTriCrRows = 64;
int64_t tri_cr_parts(int64_t nb)
{
    return std::max<int64_t>(1, std::min<int64_t>(kTriCrMaxParts, (nb + 1) / (kTriCrRows + 1)));
}
bool tri_cr_default(int M, int64_t nb, const pf_opts &o)
{
    return M == 1 && o.prec == PF_FP64 && !(o.flags & (PF_FLAG_ENLARGE | PF_FLAG_MAP_ROWS)) &&
           tri_cr_fits(nb, tri_cr_parts(nb));
}
// (scalar tridiagonal reduced levels: up to kTriMaxChain blocks, one chain in
// LDS)

// Lane mapping of a level's factor kernel: segments of E entries per lane,
// or rows (0).  One entry per lane (E = 1) spreads a chain row over M*M
// lanes and gives the lowest latency per row, which bounds the reduced
// levels; at level 0 (many partitions) fewer, wider lanes spend fewer
// instructions per partition.  With FP32 factors m = 16 uses four entries
// per lane (one wave per partition) and m = 32 the row mapping.  In FP64 the
// finest level of a block tridiagonal matrix with m = 8 (kMapMfma) and every
// level with m = 16 or 32 run their block products on the matrix cores,
// unless a mapping is asked for.
constexpr int kMapMfma = -1;
// every level of an FP64 block tridiagonal matrix with m = 32: matrix-core
// products, one partition per wave (kernels_mfma_tiles.hip)
constexpr int kMapMfma32 = -2;
// every level of an FP64 bidiagonal-plus-corner matrix with m = 16: four pivot
// blocks inverted together, the chain on the matrix cores, one partition per
// wave (kernels_mfma_tiles.hip)
constexpr int kMapMfmaB16 = -3;
// every level of an FP64 block tridiagonal matrix with m = 16: the m = 32
// kernel's scheme with one tile per product (kernels_mfma_tiles.hip)
constexpr int kMapMfma16 = -4;
// every level of an FP64 block tridiagonal matrix with m = 1 whose chains fit
// the workgroup's LDS: the segment mapping's arithmetic, rows staged through
// LDS so that loads and stores are contiguous (kernels_tri.hip)
constexpr int kMapTri = -5;

int seg_width(int M, int level, int kind, bool f32, const pf_opts &o)
{
    if (o.flags & PF_FLAG_MAP_ROWS) return 0;
    if (M == 32 && kind == PF_BTRI) return kMapMfma32;
    if (level == 0 && o.lane_entries > 0) return seg_ok(M, o.lane_entries) ? o.lane_entries : 0;
    if (M == 1 && kind == PF_BTRI && !f32 && !(o.flags & PF_FLAG_MAP_SEGMENTS)) return kMapTri;
    if (M == 16 && !(o.flags & PF_FLAG_MAP_SEGMENTS))
        return kind == PF_BABD ? kMapMfmaB16 : kMapMfma16;
    if (level == 0 && !(o.flags & (PF_FLAG_MAP_SEGMENTS | PF_FLAG_ENLARGE)) && mfma_ok(kind, M, f32, false))
        return kMapMfma;
    if (level == 0 && M == 8) return 2;   // 0.153 vs 0.156 ms per step with one entry
    for (int E = 1; E <= M; E <<= 1)
        if (seg_ok(M, E)) return E;
    return 0;
}

std::vector<PlanLevel> make_plan(int kind, int64_t nb, int M, const pf_opts &o,
                                 const SepOverrides *ovr = nullptr)
{
    std::vector<PlanLevel> out;
    const bool f32 = o.prec == PF_FP32_IR;
    int64_t cur = nb;
    int lvl = 0;
    auto explicit_at = [&](int l) -> const std::vector<int64_t> * {
        if (!ovr) return nullptr;
        auto it = ovr->find(l);
        return it == ovr->end() ? nullptr : &it->second;
    };
    if (kind == PF_BABD) {
        while (cur > 2 || explicit_at(lvl)) {
            if (const auto *sp = explicit_at(lvl)) {
                const int64_t p = (int64_t)sp->size() - 1;
                out.push_back({PF_BABD, cur, p, *sp});
                cur = p + 1;
                ++lvl;
                continue;
            }
            int64_t p;
            if (lvl == 0 && o.partitions > 0) p = o.partitions;
            else {
                const int L = lvl == 0 ? finest_chain(kind, M, f32, cur, o)
                                       : target_rows(kind, M, f32, lvl, o);
                p = (cur - 1) / (L + 1);
                p = std::max<int64_t>(p, 1);
                p = std::min<int64_t>(p, (cur - 1) / 2);
            }
            out.push_back({PF_BABD, cur, p, {}});
            cur = p + 1;
            ++lvl;
        }
        out.push_back({PF_BTRI, cur, 1, {}});
        return out;
    }
    while (true) {
        if (const auto *sp = explicit_at(lvl)) {
            const int64_t p = (int64_t)sp->size() - 1;
            out.push_back({PF_BTRI, cur, p, *sp});
            if (p == 1) break;
            cur = p - 1;
            ++lvl;
            continue;
        }
        int64_t p;
        if (lvl == 0 && o.partitions > 0) p = o.partitions;
        else if (lvl == 0 && tri_cr_default(M, cur, o)) p = tri_cr_parts(cur);
        else if (cur <= kTail || (M == 1 && lvl > 0 && cur <= kTriMaxChain)) p = 1;
        else {
            const int L = lvl == 0 ? finest_chain(kind, M, f32, cur, o)
                                   : target_rows(kind, M, f32, lvl, o);
            p = (cur + 1) / (L + 1);
            p = std::max<int64_t>(p, 2);
            p = std::min<int64_t>(p, (cur + 1) / 2);
        }
        out.push_back({PF_BTRI, cur, p, {}});
        if (p == 1) break;
        cur = p - 1;
        ++lvl;
    }
    return out;
}

size_t blk_bytes(int M, bool f32) { return (size_t)M * M * (f32 ? 4 : 8); }

// Device bytes of the factor of a plan (without the solve workspace).
size_t plan_bytes(const std::vector<PlanLevel> &plan, int M, int m, const pf_opts &o)
{
    size_t b = 0;
    const size_t bd = (size_t)M * M * 8;
    for (size_t l = 0; l < plan.size(); ++l) {
        const bool f32 = (l == 0 && o.prec == PF_FP32_IR);
        const PlanLevel &L = plan[l];
        const int nfac = (L.kind == PF_BTRI) ? 4 : 2;
        b += (size_t)nfac * (size_t)L.nb * blk_bytes(M, f32);
        if (L.kind == PF_BTRI && L.p > 1) b += 4 * (size_t)(L.p - 1) * bd;
        if (L.kind == PF_BABD) b += (size_t)(2 * L.p + 2) * bd;
    }
    if (M != m) b += 3 * (size_t)plan[0].nb * bd;  // padded copy of A
    return b + 256;
}

// Device memory of a handle: stream-ordered allocations of its own, or
// 256-byte aligned slices of a batch's arena.  A counting arena only adds up
// sizes (the pointers it hands out are never dereferenced: no launch happens
// while counting).
hipError_t dalloc(pf_factor_s *F, void **p, size_t bytes, std::vector<DevBlock> &list)
{
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    if (F->arena) {
        Arena &ar = *F->arena;
        const size_t off = (ar.off + 255) & ~(size_t)255;
        if (!ar.counting && off + bytes > ar.cap) return hipErrorOutOfMemory;
        *p = ar.counting ? (void *)(uintptr_t)(4096 + off) : (void *)(ar.base + off);
        ar.off = off + bytes;
        return hipSuccess;
    }
    hipError_t e = dev_alloc(F->al, p, bytes, F->stream);
    if (e != hipSuccess) { *p = nullptr; return e; }
    list.push_back({*p, bytes});
    return hipSuccess;
}

void free_list(pf_factor_s *F, std::vector<DevBlock> &list)
{
    for (const DevBlock &b : list) dev_free(F->al, b.p, b.bytes, F->stream);
    list.clear();
}

int check_matrix(const pf_matrix *A)
{
    if (!A) return -1;
    if (A->kind != PF_BTRI && A->kind != PF_BABD) return -1;
    if (A->m < 1 || A->nb < 2 || !A->D || !A->Lo) return -1;
    if (A->kind == PF_BTRI && (!A->Up || A->C)) return -1;
    if (A->kind == PF_BABD && (A->Up || !A->C)) return -1;
    if (A->m > kMaxM) return PF_EUNSUPPORTED;
    return 0;
}

pf_opts resolve_opts(const pf_opts *o)
{
    pf_opts r{};
    if (o) r = *o;
    if (r.max_refine <= 0) r.max_refine = 10;
    if (!(r.tol > 0)) r.tol = 1e-12;
    return r;
}

int check_opts(const pf_matrix *A, const pf_opts &o)
{
    if (o.prec != PF_FP64 && o.prec != PF_FP32_IR) return -2;
    if (o.partitions < 0 || o.block_rows < 0 || o.coarse_rows < 0 || o.lane_entries < 0) return -2;
    if (o.lane_entries > 0 && !(o.flags & PF_FLAG_MAP_ROWS) &&
        !seg_ok(padded_block(A->m), o.lane_entries))
        return -2;
    if (o.partitions > 0) {
        const int64_t pmax = (A->kind == PF_BTRI) ? (A->nb + 1) / 2 : (A->nb - 1) / 2;
        if (o.partitions > pmax && !(A->kind == PF_BABD && A->nb == 2)) return -2;
    }
    return 0;
}

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) {                     \
            g_last_hip = (int)e_;                   \
            return PF_EHIP;                         \
        }                                           \
    } while (0)

// Run one launch, bracketed by HIP events on its stream when profiling.
template <class Fn>
hipError_t prof_launch(pf_factor_s *F, bool factor, int phase, int level, hipStream_t s, Fn fn)
{
    if (!F->prof) return fn();
    auto &list = factor ? F->prof_fac : F->prof_sol;
    size_t &n = factor ? F->prof_fac_n : F->prof_sol_n;
    if (n >= list.size()) {
        pf_factor_s::ProfSlot sl;
        if (hipEventCreate(&sl.a) != hipSuccess || hipEventCreate(&sl.b) != hipSuccess)
            return hipErrorOutOfMemory;
        list.push_back(sl);
    }
    auto &sl = list[n++];
    sl.phase = phase;
    sl.level = level;
    // the launch stamps its kernel's own start and end into the events
    LaunchTiming &t = launch_timing();
    t.start = sl.a;
    t.stop = sl.b;
    hipError_t e = fn();
    if (t.start) {   // nothing was launched: mark the point in the stream
        t.start = t.stop = nullptr;
        if (e == hipSuccess) e = hipEventRecord(sl.a, s);
        if (e == hipSuccess) e = hipEventRecord(sl.b, s);
    }
    return e;
}

// Kernel arguments of the factorization of level l.
LevelArgs level_args(const pf_factor_s *F, size_t l)
{
    const Level &L = F->lv[l];
    LevelArgs a{};
    a.nb = L.nb; a.p = L.p;
    a.D = L.D; a.Dadd = L.Dadd; a.Lo = L.Lo; a.Up = L.Up; a.C = L.C;
    a.E = L.E; a.R = L.R; a.Z = L.Z; a.X = L.X;
    a.nD = L.nD; a.nDadd = L.nDadd; a.nLo = L.nLo; a.nUp = L.nUp; a.nC = L.nC;
    a.status = F->d_status;
    a.dump = F->d_dump;
    a.zero = F->d_zero;
    a.level = (int)l;
    a.sep = L.d_sep;
    if (F->d_badlist) {
        a.tau = L.f32 ? 0x1p-20 : 0x1p-40;
        a.badlist = F->d_badlist;
        a.badcount = (unsigned *)(F->d_badlist + kBadCap);
        a.badcap = kBadCap;
    }
    return a;
}

// Kernel arguments of every level of one solve: F0/Y0 are the (padded when
// M != m) right-hand side and solution of level 0, the other levels use the
// handle's workspace.
std::vector<SolveArgs> solve_args(const pf_factor_s *F, int nrhs, const double *F0, int64_t ld0f,
                                  double *Y0, int64_t ld0y)
{
    const int M = F->M;
    const size_t L = F->lv.size();
    std::vector<SolveArgs> args(L);
    for (size_t l = 0; l < L; ++l) {
        const Level &lv = F->lv[l];
        SolveArgs &a = args[l];
        a = SolveArgs{};
        a.nb = lv.nb;
        a.dump = (double *)F->d_dump;
        a.zero = F->d_zero;
        a.p = lv.p;
        a.sep = lv.d_sep;
        a.nrhs = nrhs;
        a.Lo = lv.Lo;
        a.E = lv.E; a.R = lv.R; a.Z = lv.Z; a.X = lv.X;
        if (l == 0) {
            a.F = F0; a.ldf = ld0f; a.Fadd = nullptr; a.Y = Y0; a.ldy = ld0y;
        } else {
            a.F = F->wsF[l];
            a.Fadd = F->wsFadd[l];
            a.ldf = lv.nb * M;
            a.Y = F->wsY[l];
            a.ldy = lv.nb * M;
        }
        if (l + 1 < L) {
            a.nF = F->wsF[l + 1];
            a.nFadd = F->wsFadd[l + 1];
            a.ldn = F->lv[l + 1].nb * M;
            a.Xsep = F->wsY[l + 1];
        } else {
            a.ldn = 1;
        }
    }
    return args;
}

// Level-0 matrix copied into the instantiated block size (M != m).
hipError_t pad_matrix(pf_factor_s *F, hipStream_t s)
{
    const pf_matrix &A0 = F->A;
    hipError_t e = launch_pad_blocks(A0.m, F->M, A0.nb, A0.D, F->padD, 1.0, s);
    if (e == hipSuccess) e = launch_pad_blocks(A0.m, F->M, A0.nb - 1, A0.Lo, F->padLo, 0.0, s);
    if (e == hipSuccess && F->padUp)
        e = launch_pad_blocks(A0.m, F->M, A0.nb - 1, A0.Up, F->padUp, 0.0, s);
    if (e == hipSuccess && F->padC) e = launch_pad_blocks(A0.m, F->M, 1, A0.C, F->padC, 0.0, s);
    return e;
}

hipError_t launch_factor_levels(pf_factor_s *F, hipStream_t s)
{
    F->prof_fac_n = 0;
    hipError_t e = launch_fill_u64(F->d_status, 1, ~0ull, s);
    if (e != hipSuccess) return e;
    if (F->d_badlist &&
        (e = launch_fill_u64(F->d_badlist + kBadCap, 1, 0ull, s)) != hipSuccess)
        return e;
    if (F->M != F->m && (e = pad_matrix(F, s)) != hipSuccess) return e;
    for (size_t l = 0; l < F->lv.size(); ++l) {
        const Level &L = F->lv[l];
        const LevelArgs a = level_args(F, l);
        e = prof_launch(F, true, 0, (int)l, s, [&] {
            if (L.seg == kMapMfma) return launch_mfma_factor(a, nullptr, s);
            if (L.seg == kMapMfma32) return launch_mfma32_factor(a, L.f32, s);
            if (L.seg == kMapMfma16) return launch_mfma16_factor(a, nullptr, L.f32, s);
            if (L.seg == kMapMfmaB16) return launch_mfma_babd16_factor(a, nullptr, L.f32, s);
            if (L.seg == kMapTri) return launch_tri_factor(a, nullptr, s);
            if (L.seg) return launch_seg_factor(L.kind, F->M, L.seg, L.f32, a, nullptr, s);
            return (L.kind == PF_BTRI) ? launch_btri_factor(F->M, L.f32, a, s)
                                       : launch_babd_factor(F->M, L.f32, a, s);
        });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int ensure_workspace(pf_factor_s *F, int nrhs)
{
    if (nrhs <= F->rhs_cap) return 0;
    hipError_t e_;
    free_list(F, F->ws_allocs);
    // a handle carved from a batch arena grows its workspace in memory of
    // its own (the arena is sized for the batch's right-hand sides only)
    Arena *const ar = F->arena;
    if (ar && !ar->counting && F->rhs_cap > 0) F->arena = nullptr;
    struct Restore {
        pf_factor_s *F;
        Arena *ar;
        ~Restore() { F->arena = ar; }
    } restore{F, ar};
    const int cap = std::max(nrhs, 1);
    const size_t L = F->lv.size();
    F->wsF.assign(L, nullptr);
    F->wsFadd.assign(L, nullptr);
    F->wsY.assign(L, nullptr);
    for (size_t l = 1; l < L; ++l) {
        const size_t bytes = (size_t)F->lv[l].nb * F->M * cap * sizeof(double);
        void *p;
        if ((e_ = dalloc(F, &p, bytes, F->ws_allocs)) != hipSuccess) return alloc_status(e_);
        F->wsF[l] = (double *)p;
        if (F->lv[l - 1].kind == PF_BTRI) {
            if ((e_ = dalloc(F, &p, bytes, F->ws_allocs)) != hipSuccess) return alloc_status(e_);
            F->wsFadd[l] = (double *)p;
        }
        if ((e_ = dalloc(F, &p, bytes, F->ws_allocs)) != hipSuccess) return alloc_status(e_);
        F->wsY[l] = (double *)p;
    }
    const size_t nP = (size_t)F->nb * F->M * cap * sizeof(double);
    const size_t n = (size_t)F->nb * F->m * cap * sizeof(double);
    void *p;
    if (F->M != F->m) {
        if ((e_ = dalloc(F, &p, nP, F->ws_allocs)) != hipSuccess) return alloc_status(e_);
        F->wsPadF = (double *)p;
        if ((e_ = dalloc(F, &p, nP, F->ws_allocs)) != hipSuccess) return alloc_status(e_);
        F->wsPadX = (double *)p;
    }
    if (F->opts.prec == PF_FP32_IR) {   // residual and correction of the refinement
        if ((e_ = dalloc(F, &p, n, F->ws_allocs)) != hipSuccess) return alloc_status(e_);
        F->wsR = (double *)p;
        if ((e_ = dalloc(F, &p, n, F->ws_allocs)) != hipSuccess) return alloc_status(e_);
        F->wsD = (double *)p;
    }
    if ((e_ = dalloc(F, &p, 3 * (size_t)cap * sizeof(unsigned long long), F->ws_allocs)) !=
        hipSuccess)
        return alloc_status(e_);
    F->d_norms = (unsigned long long *)p;
    F->rhs_cap = cap;
    return 0;
}

// One pass of the method over nrhs right-hand sides: x = (FTG)^{-1} f.
int run_solve(pf_factor_s *F, int nrhs, const double *f, int64_t ldf, double *x, int64_t ldx,
              hipStream_t s)
{
    const int M = F->M;
    const size_t L = F->lv.size();
    const double *F0 = f;
    int64_t ld0f = ldf, ld0y = ldx;
    double *Y0 = x;
    if (M != F->m) {
        const int64_t ldp = (int64_t)F->nb * M;
        HIPCHK(launch_pad_rhs(F->m, M, F->nb, nrhs, f, ldf, F->wsPadF, ldp, true, s));
        F0 = F->wsPadF;
        Y0 = F->wsPadX;
        ld0f = ld0y = ldp;
    }
    const std::vector<SolveArgs> args = solve_args(F, nrhs, F0, ld0f, Y0, ld0y);
    F->prof_sol_n = 0;
    for (size_t l = 0; l < L; ++l) {
        const Level &lv = F->lv[l];
        HIPCHK(prof_launch(F, false, 1, (int)l, s, [&] {
            return lv.kind != PF_BTRI ? launch_babd_fwd(M, lv.f32, args[l], s)
                   : (lv.seg == kMapTri && args[l].nrhs == 1) ? launch_tri_fwd(args[l], s)
                                                              : launch_btri_fwd(M, lv.f32, args[l], s);
        }));
    }
    for (size_t l = L; l-- > 0;) {
        const Level &lv = F->lv[l];
        HIPCHK(prof_launch(F, false, 2, (int)l, s, [&] {
            return lv.kind != PF_BTRI ? launch_babd_bwd(M, lv.f32, args[l], s)
                   : (lv.seg == kMapTri && args[l].nrhs == 1) ? launch_tri_bwd(args[l], s)
                                                              : launch_btri_bwd(M, lv.f32, args[l], s);
        }));
    }
    if (M != F->m)
        HIPCHK(launch_pad_rhs(F->m, M, F->nb, nrhs, F->wsPadX, (int64_t)F->nb * M, x, ldx, false,
                              s));
    return 0;
}

// Factor-and-solve in one pass per level (every level on the segment mapping,
// 1 <= nrhs <= M): the factor kernels also sweep the right-hand sides
// forward, then the back substitution runs up the levels as in run_solve.
// Factor-and-solve of a small scalar tridiagonal system (one right-hand
// side) in one launch: the finest level's partitions by local cyclic
// reduction, the reduced system across one wave, the back substitution.  The
// launch sets the status word itself; the stored factors are left behind
// (pf_solve refactors first).
int run_tri_cr(pf_factor_s *F, const double *f, double *x, hipStream_t s)
{
    const pf_matrix &A = F->A;
    F->prof_fac_n = 0;
    F->prof_sol_n = 0;
    HIPCHK(prof_launch(F, true, 3, 0, s, [&] {
        return launch_tri_cr_whole(A.nb, F->lv[0].p, A.D, A.Lo, A.Up, f, x, F->d_status, s);
    }));
    F->factors_stale = true;
    return 0;
}

bool fused_ok(const pf_factor_s *F, int nrhs)
{
    if (nrhs < 1 || nrhs > F->M) return false;
    for (const Level &L : F->lv)
        if (L.seg == 0 || L.seg == kMapMfma32) return false;
    return true;
}

int run_factor_solve(pf_factor_s *F, int nrhs, const double *f, int64_t ldf, double *x,
                     int64_t ldx, hipStream_t s)
{
    const int M = F->M;
    const size_t L = F->lv.size();
    F->prof_fac_n = 0;
    F->prof_sol_n = 0;
    HIPCHK(launch_fill_u64(F->d_status, 1, ~0ull, s));
    if (F->d_badlist) HIPCHK(launch_fill_u64(F->d_badlist + kBadCap, 1, 0ull, s));
    const double *F0 = f;
    int64_t ld0f = ldf, ld0y = ldx;
    double *Y0 = x;
    if (M != F->m) {
        HIPCHK(pad_matrix(F, s));
        const int64_t ldp = (int64_t)F->nb * M;
        HIPCHK(launch_pad_rhs(F->m, M, F->nb, nrhs, f, ldf, F->wsPadF, ldp, true, s));
        F0 = F->wsPadF;
        Y0 = F->wsPadX;
        ld0f = ld0y = ldp;
    }
    const std::vector<SolveArgs> args = solve_args(F, nrhs, F0, ld0f, Y0, ld0y);
    for (size_t l = 0; l < L; ++l) {
        const Level &lv = F->lv[l];
        const LevelArgs a = level_args(F, l);
        HIPCHK(prof_launch(F, true, 3, (int)l, s, [&] {
            if (lv.seg == kMapMfma) return launch_mfma_factor(a, &args[l], s);
            if (lv.seg == kMapMfmaB16) return launch_mfma_babd16_factor(a, &args[l], lv.f32, s);
            if (lv.seg == kMapMfma16) return launch_mfma16_factor(a, &args[l], lv.f32, s);
            if (lv.seg == kMapTri) return launch_tri_factor(a, &args[l], s);
            return launch_seg_factor(lv.kind, M, lv.seg, lv.f32, a, &args[l], s);
        }));
    }
    for (size_t l = L; l-- > 0;) {
        const Level &lv = F->lv[l];
        HIPCHK(prof_launch(F, false, 2, (int)l, s, [&] {
            return lv.kind != PF_BTRI ? launch_babd_bwd(M, lv.f32, args[l], s)
                   : (lv.seg == kMapTri && args[l].nrhs == 1) ? launch_tri_bwd(args[l], s)
                                                              : launch_btri_bwd(M, lv.f32, args[l], s);
        }));
    }
    if (M != F->m)
        HIPCHK(launch_pad_rhs(F->m, M, F->nb, nrhs, F->wsPadX, (int64_t)F->nb * M, x, ldx, false,
                              s));
    return 0;
}

double bits_to_double(unsigned long long b)
{
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

// eta per right-hand side from the norms buffer; returns the max over columns.
// The residual r = f - A x with its norms, and ||A||, queued on s into the
// host words h (3 nrhs + 1: per column ||r||, ||x||, ||f||, then ||A||).
int queue_residual_norms(pf_factor_s *F, int nrhs, const double *f, int64_t ldf, const double *x,
                         int64_t ldx, double *r, int64_t ldr, hipStream_t s,
                         unsigned long long *h)
{
    const pf_matrix &A = F->A;
    HIPCHK(launch_fill_u64(F->d_norms, 3 * nrhs, 0ull, s));
    HIPCHK(launch_fill_u64(F->d_norm, 1, 0ull, s));
    HIPCHK(launch_residual(A.kind, A.m, A.nb, A.D, A.Lo, A.Up, A.C, nrhs, f, ldf, x, ldx, r, ldr,
                           F->d_norms, F->d_norm, s));
    HIPCHK(hipMemcpyAsync(h, F->d_norms, 3 * nrhs * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h + 3 * nrhs, F->d_norm, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s));
    return 0;
}

// eta (max over columns) from the words queue_residual_norms filled
double eta_of(const unsigned long long *h, int nrhs)
{
    const double na = bits_to_double(h[3 * nrhs]);
    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c) {
        const double nr = bits_to_double(h[3 * c]), nx = bits_to_double(h[3 * c + 1]),
                     nf = bits_to_double(h[3 * c + 2]);
        const double den = na * nx + nf;
        double e = den > 0 ? nr / den : (nr > 0 ? INFINITY : 0.0);
        if (std::isnan(e)) e = INFINITY;
        worst = std::max(worst, e);
    }
    return worst;
}

int compute_eta(pf_factor_s *F, int nrhs, const double *f, int64_t ldf, const double *x,
                int64_t ldx, double *r, int64_t ldr, hipStream_t s, double *eta_out)
{
    std::vector<unsigned long long> h(3 * nrhs + 1);
    const int rc = queue_residual_norms(F, nrhs, f, ldf, x, ldx, r, ldr, s, h.data());
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s));
    *eta_out = eta_of(h.data(), nrhs);
    return 0;
}

// The handle's device status word into info (PF_EHIP when it cannot be read).
void read_status(pf_factor_s *F, pf_info *info)
{
    unsigned long long st = ~0ull;
    const hipError_t e = hipMemcpy(&st, F->d_status, sizeof st, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        info->status = PF_EHIP;
        info->bad_level = 0;
        info->bad_block = -1;
        return;
    }
    if (st != ~0ull) {
        info->status = PF_ESINGULAR;
        info->bad_level = (int32_t)(st >> 40);
        info->bad_block = (int64_t)(st & ((1ull << 40) - 1));
    } else {
        info->status = PF_OK;
        info->bad_level = 0;
        info->bad_block = -1;
    }
}

}  // namespace

extern "C" {

const char *pf_strerror(int code)
{
    if (code < 0) return "invalid argument";
    switch (code) {
    case PF_OK: return "success";
    case PF_ESINGULAR: return "exactly zero pivot in a pivot block";
    case PF_ENOCONV: return "iterative refinement did not converge";
    case PF_ENOMEM: return "device allocation failed";
    case PF_EHIP: return "HIP runtime error";
    case PF_EUNSUPPORTED: return "block size not supported";
    case PF_ETOOBIG: return "system does not fit the library's static workspace";
    default: return "unknown error";
    }
}

int pf_set_allocator(pf_alloc_fn alloc, pf_free_fn free_fn, void *ctx)
{
    if ((alloc == nullptr) != (free_fn == nullptr)) return alloc ? -2 : -1;
    g_allocator = Allocator{alloc, free_fn, alloc ? ctx : nullptr};
    return 0;
}

int pf_last_hip_error(void) { return g_last_hip; }

size_t pf_factor_bytes(const pf_matrix *A, const pf_opts *opts)
{
    if (check_matrix(A) != 0) return 0;
    const pf_opts o = resolve_opts(opts);
    if (check_opts(A, o) != 0) return 0;
    const int M = padded_block(A->m);
    return plan_bytes(make_plan(A->kind, A->nb, M, o), M, A->m, o);
}

size_t pf_solve_bytes_per_rhs(const pf_matrix *A, const pf_opts *opts)
{
    if (check_matrix(A) != 0) return 0;
    const pf_opts o = resolve_opts(opts);
    if (check_opts(A, o) != 0) return 0;
    const int M = padded_block(A->m);
    const auto plan = make_plan(A->kind, A->nb, M, o);
    size_t b = 0;
    for (size_t l = 1; l < plan.size(); ++l) b += 3 * (size_t)plan[l].nb * M * 8;
    if (M != A->m) b += 2 * (size_t)A->nb * M * 8;
    if (o.prec == PF_FP32_IR) b += 2 * (size_t)A->nb * A->m * 8;   // residual, correction
    b += 24;
    return b;
}

}  // extern "C"

namespace {

// Allocate and wire a handle for an already validated matrix: plan, factor
// storage, reduced systems, status words.  No kernel runs here.  With an
// arena the memory comes from it; with shared scratch (a batch) the handle
// uses it for its dump and zero areas instead of its own.
int factor_setup(const pf_matrix *A, const pf_opts &o, hipStream_t s, Arena *arena,
                 void *shared_scratch, pf_factor_s **out, const SepOverrides *ovr = nullptr)
{
    pf_factor_s *F = new pf_factor_s();
    F->al = g_allocator;
    F->A = *A;
    F->opts = o;
    F->m = A->m;
    F->M = padded_block(A->m);
    F->nb = A->nb;
    F->stream = s;
    F->arena = arena;
    const int M = F->M;
    const size_t bd = (size_t)M * M * sizeof(double);
    auto fail = [&](int code) {
        free_list(F, F->allocs);
        if (!arena) hipStreamSynchronize(s);
        delete F;
        return code;
    };
    void *p;
    hipError_t e_;
    if ((e_ = dalloc(F, &p, 2 * sizeof(unsigned long long), F->allocs)) != hipSuccess)
        return fail(alloc_status(e_));
    F->d_status = (unsigned long long *)p;
    F->d_norm = F->d_status + 1;
    if (shared_scratch) F->d_dump = shared_scratch;
    else if ((e_ = dalloc(F, &F->d_dump, kDumpBytes + kZeroBytes, F->allocs)) != hipSuccess)
        return fail(alloc_status(e_));
    F->d_zero = (const double *)((char *)F->d_dump + kDumpBytes);

    // level-0 matrix (padded to an instantiated block size if needed; the
    // padding itself runs in launch_factor_levels so refactor redoes it)
    const double *D0 = A->D, *Lo0 = A->Lo, *Up0 = A->Up, *C0 = A->C;
    if (M != A->m) {
        if ((e_ = dalloc(F, &p, A->nb * bd, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
        F->padD = (double *)p;
        if ((e_ = dalloc(F, &p, (A->nb - 1) * bd, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
        F->padLo = (double *)p;
        D0 = F->padD;
        Lo0 = F->padLo;
        if (A->kind == PF_BTRI) {
            if ((e_ = dalloc(F, &p, (A->nb - 1) * bd, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
            F->padUp = (double *)p;
            Up0 = F->padUp;
        } else {
            if ((e_ = dalloc(F, &p, bd, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
            F->padC = (double *)p;
            C0 = F->padC;
        }
    }

    const auto plan = make_plan(A->kind, A->nb, M, o, ovr);
    F->lv.resize(plan.size());
    F->tri_cr = A->kind == PF_BTRI && M == 1 && A->m == 1 && o.prec == PF_FP64 &&
                !(o.flags & (PF_FLAG_ENLARGE | PF_FLAG_MAP_ROWS | PF_FLAG_ETA |
                             PF_FLAG_MAP_SEGMENTS)) && !ovr &&
                tri_cr_fits(A->nb, plan[0].p);
    const bool counting = arena && arena->counting;
    if (o.flags & PF_FLAG_ENLARGE) {
        if ((e_ = dalloc(F, &p, kBadCap * sizeof(unsigned long long) + 256, F->allocs)) != hipSuccess)
            return fail(alloc_status(e_));
        F->d_badlist = (unsigned long long *)p;
    }
    for (size_t l = 0; l < plan.size(); ++l) {
        Level &L = F->lv[l];
        L.kind = plan[l].kind;
        L.nb = plan[l].nb;
        L.p = plan[l].p;
        L.f32 = (l == 0 && o.prec == PF_FP32_IR);
        L.seg = seg_width(M, (int)l, L.kind, L.f32, o);
        if (L.seg == kMapTri && !tri_fits(L.nb, L.p)) L.seg = 1;
        if (!plan[l].seps.empty()) {
            // explicit boundaries: the kernels that follow them (not the
            // LDS-staged scalar chains, whose staging assumes the balanced rule)
            L.seps = plan[l].seps;
            if (L.seg == kMapTri) L.seg = 1;
            const size_t sb = L.seps.size() * sizeof(int64_t);
            if ((e_ = dalloc(F, &p, sb, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
            L.d_sep = (int64_t *)p;
            if (!counting &&
                (e_ = hipMemcpyAsync(L.d_sep, L.seps.data(), sb, hipMemcpyHostToDevice, s)) !=
                    hipSuccess)
                return fail(alloc_status(e_));
        }
        if (l == 0) {
            L.D = D0; L.Lo = Lo0;
            if (A->kind == PF_BTRI) L.Up = Up0;
            else if (L.kind == PF_BABD) L.C = C0;
            else L.Up = C0;   // a two-block BABD is block tridiagonal with Up = corner
        } else {
            const Level &P = F->lv[l - 1];
            L.D = P.nD;
            L.Dadd = P.nDadd;
            L.Lo = P.nLo;
            if (P.kind == PF_BTRI) L.Up = P.nUp;
            else if (L.kind == PF_BABD) L.C = P.nC;
            else L.Up = P.nC;
        }
        const size_t fb = (size_t)L.nb * blk_bytes(M, L.f32);
        if ((e_ = dalloc(F, &L.E, fb, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
        if ((e_ = dalloc(F, &L.Z, fb, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
        if (L.kind == PF_BTRI) {
            if ((e_ = dalloc(F, &L.R, fb, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
            if ((e_ = dalloc(F, &L.X, fb, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
            if (L.p > 1) {
                const size_t rb = (size_t)(L.p - 1) * bd;
                if ((e_ = dalloc(F, &p, rb, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
                L.nD = (double *)p;
                if ((e_ = dalloc(F, &p, rb, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
                L.nDadd = (double *)p;
                if ((e_ = dalloc(F, &p, rb, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
                L.nLo = (double *)p;
                if ((e_ = dalloc(F, &p, rb, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
                L.nUp = (double *)p;
            }
        } else {
            if ((e_ = dalloc(F, &p, (size_t)(L.p + 1) * bd, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
            L.nD = (double *)p;
            if ((e_ = dalloc(F, &p, (size_t)L.p * bd, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
            L.nLo = (double *)p;
            if ((e_ = dalloc(F, &p, bd, F->allocs)) != hipSuccess) return fail(alloc_status(e_));
            L.nC = (double *)p;
        }
    }
    *out = F;
    return 0;
}

// A handle whose memory (factors, reduced systems, status, scratch and the
// solve workspace for nrhs right-hand sides) is one stream-ordered device
// allocation: the sizes come from a counting pass through the same set-up
// code.  One allocation instead of dozens keeps the host cost of a new
// factorization low (a serving request pays it every time).
int factor_setup_private(const pf_matrix *A, const pf_opts &o, hipStream_t s, int nrhs,
                         pf_factor_s **out, const Allocator *al = nullptr,
                         const SepOverrides *ovr = nullptr)
{
    Arena count;
    count.counting = true;
    pf_factor_s *T = nullptr;
    int rc = factor_setup(A, o, s, &count, nullptr, &T, ovr);
    if (rc) return rc;
    rc = ensure_workspace(T, nrhs);
    delete T;
    if (rc) return rc;
    Arena *ar = new Arena();
    ar->cap = count.off + 256;
    ar->refs = 1;
    ar->al = al ? *al : g_allocator;
    const hipError_t e = dev_alloc(ar->al, (void **)&ar->base, ar->cap, s);
    if (e != hipSuccess) {
        delete ar;
        return alloc_status(e);
    }
    pf_factor_s *F = nullptr;
    if ((rc = factor_setup(A, o, s, ar, nullptr, &F, ovr)) || (rc = ensure_workspace(F, nrhs))) {
        if (F) {
            F->arena = nullptr;
            delete F;
        }
        dev_free(ar->al, ar->base, ar->cap, s);
        delete ar;
        return rc;
    }
    *out = F;
    return 0;
}

// Partition boundaries of a level as a list (balanced rule, or explicit).
std::vector<int64_t> level_bounds(const Level &L)
{
    if (!L.seps.empty()) return L.seps;
    std::vector<int64_t> b(L.p + 1);
    const bool btri = L.kind == PF_BTRI;
    const int64_t nint = btri ? L.nb - (L.p - 1) : L.nb - (L.p + 1);
    const int64_t q = nint / L.p, rem = nint % L.p;
    b[0] = btri ? -1 : 0;
    for (int64_t i = 0; i < L.p; ++i) b[i + 1] = b[i] + q + (i < rem ? 1 : 0) + 1;
    return b;   // BTRI: b[p] = nb; BABD: b[p] = nb - 1
}

constexpr int kMaxEnlargePasses = 32;

// Factorization with the reduced system enlarged where the local
// eliminations fail (Sec. 2, the modified factorization after eq. (redmatr)):
// a pass factors every level and lists, per failing partition, its first
// pivot block that is singular or ill-conditioned; those block rows of the
// lowest failing level become separators (the partition's elimination stops
// before them and they enter the reduced system), that level is planned
// again with the enlarged separator list and the levels above it anew, and
// the next pass factors again, until no pivot block fails or the passes run
// out (the status then reports the first failing block).  Synchronizes s.
int factor_enlarged(const pf_matrix *A, const pf_opts &o, hipStream_t s, pf_factor_t *out)
{
    SepOverrides ovr;
    pf_factor_s *F = nullptr;
    for (int pass = 0;; ++pass) {
        int rc = factor_setup_private(A, o, s, 1, &F, nullptr, &ovr);
        if (rc) return rc;
        hipError_t e = launch_fill_u64((unsigned long long *)F->d_zero, kZeroBytes / 8, 0ull, s);
        if (e == hipSuccess) e = launch_factor_levels(F, s);
        std::vector<unsigned long long> h(kBadCap + 1);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h.data(), F->d_badlist, (kBadCap + 1) * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            pf_destroy(F);
            return PF_EHIP;
        }
        const unsigned cnt = std::min<unsigned>((unsigned)h[kBadCap], (unsigned)kBadCap);
        // In the bidiagonal-plus-corner form the reduced matrix (eq.
        // (redmatr1)) keeps each separator's own diagonal block (no
        // contribution is added to it), so a failing block would fail again
        // on every reduced level: there the pass only detects and reports.
        if (cnt == 0 || A->kind == PF_BABD || pass + 1 >= kMaxEnlargePasses) break;
        std::vector<unsigned long long> codes(h.begin(), h.begin() + cnt);
        std::sort(codes.begin(), codes.end());
        codes.erase(std::unique(codes.begin(), codes.end()), codes.end());
        const int lvl = (int)(codes.front() >> 40);
        std::vector<int64_t> b = level_bounds(F->lv[lvl]);
        for (unsigned long long c : codes)
            if ((int)(c >> 40) == lvl) b.push_back((int64_t)(c & ((1ull << 40) - 1)));
        std::sort(b.begin(), b.end());
        b.erase(std::unique(b.begin(), b.end()), b.end());
        ovr[lvl] = b;
        ovr.erase(ovr.upper_bound(lvl), ovr.end());
        pf_destroy(F);
        F = nullptr;
    }
    *out = F;
    return 0;
}

}  // namespace

extern "C" {

int pf_factor(const pf_matrix *A, const pf_opts *opts, void *stream, pf_factor_t *out)
{
    if (!out) return -4;
    *out = nullptr;
    int rc = check_matrix(A);
    if (rc) return rc;
    pf_opts o = resolve_opts(opts);
    if ((rc = check_opts(A, o))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (o.flags & PF_FLAG_AUTOTUNE) {
        pf_opts t{};
        if ((rc = tuned_opts(A, o, 1, s, &t))) return rc;
        o = resolve_opts(&t);
    }
    if (o.flags & PF_FLAG_ENLARGE) return factor_enlarged(A, o, s, out);
    pf_factor_s *F = nullptr;
    if ((rc = factor_setup_private(A, o, s, 1, &F))) return rc;
    hipError_t e = launch_fill_u64((unsigned long long *)F->d_zero, kZeroBytes / 8, 0ull, s);
    if (e == hipSuccess) e = launch_factor_levels(F, s);
    if (e != hipSuccess) {
        pf_destroy(F);
        return PF_EHIP;
    }
    *out = F;
    return 0;
}

int pf_refactor(pf_factor_t F, void *stream)
{
    if (!F) return -1;
    hipStream_t s = stream ? (hipStream_t)stream : F->stream;
    if (launch_factor_levels(F, s) != hipSuccess) return PF_EHIP;
    F->factors_stale = false;
    return 0;
}

int pf_profile_enable(pf_factor_t F, int enable)
{
    if (!F) return -1;
    F->prof = enable != 0;
    return 0;
}

int pf_profile_read(pf_factor_t F, int32_t max, int32_t *phase, int32_t *level, float *ms)
{
    if (!F) return -1;
    if (hipDeviceSynchronize() != hipSuccess) return PF_EHIP;
    int n = 0;
    for (int which = 0; which < 2; ++which) {
        const auto &list = which == 0 ? F->prof_fac : F->prof_sol;
        const size_t cnt = which == 0 ? F->prof_fac_n : F->prof_sol_n;
        for (size_t i = 0; i < cnt; ++i, ++n) {
            if (n >= max) continue;
            float t = 0.f;
            if (hipEventElapsedTime(&t, list[i].a, list[i].b) != hipSuccess) t = -1.f;
            if (phase) phase[n] = list[i].phase;
            if (level) level[n] = list[i].level;
            if (ms) ms[n] = t;
        }
    }
    return n;
}

int pf_residual(const pf_matrix *A, int32_t nrhs, const double *f, int64_t ldf, const double *x,
                int64_t ldx, double *r, int64_t ldr, void *stream, double *norms)
{
    int rc = check_matrix(A);
    if (rc) return rc < 0 ? -1 : rc;
    const int64_t n = A->nb * A->m;
    if (nrhs < 0) return -2;
    if (nrhs > 0 && !f) return -3;
    if (ldf < n) return -4;
    if (nrhs > 0 && !x) return -5;
    if (ldx < n) return -6;
    if (r && ldr < n) return -8;
    if (!norms) return -10;
    hipStream_t s = (hipStream_t)stream;
    const size_t words = 3 * (size_t)nrhs + 1;
    unsigned long long *d = nullptr;
    hipError_t e = dev_alloc(g_allocator, (void **)&d, words * sizeof *d, s);
    if (e != hipSuccess) return alloc_status(e);
    std::vector<unsigned long long> h(words);
    e = launch_fill_u64(d, (int64_t)words, 0ull, s);
    if (e == hipSuccess)
        e = launch_residual(A->kind, A->m, A->nb, A->D, A->Lo, A->Up, A->C, nrhs, f, ldf, x, ldx,
                            r, r ? ldr : n, d, d + 3 * nrhs, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), d, words * sizeof *d, hipMemcpyDeviceToHost, s);
    dev_free(g_allocator, d, words * sizeof *d, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        return PF_EHIP;
    }
    for (size_t i = 0; i < words; ++i) norms[i] = bits_to_double(h[i]);
    return 0;
}

int pf_sync_status(pf_factor_t F, pf_info *info)
{
    if (!F) return -1;
    if (!info) return -2;
    if (hipStreamSynchronize(F->stream) != hipSuccess) return PF_EHIP;
    std::memset(info, 0, sizeof *info);
    info->eta = -1.0;
    read_status(F, info);
    return info->status;
}

}  // extern "C"

namespace {

// A solve call: x = A^{-1} f by `first` (a pass of the method over the
// right-hand sides: run_solve, or run_factor_solve that also refactors),
// then, for PF_FP32_IR, FP64 refinement with correction solves.
template <class First>
int solve_call(pf_factor_s *F, int32_t nrhs, const double *f, int64_t ldf, double *x, int64_t ldx,
               void *stream, pf_info *info, First first)
{
    if (!F) return -1;
    if (nrhs < 0) return -2;
    const int64_t n = F->nb * F->m;
    if (nrhs > 0 && !f) return -3;
    if (ldf < n) return -4;
    if (nrhs > 0 && !x) return -5;
    if (ldx < n) return -6;
    hipStream_t s = stream ? (hipStream_t)stream : F->stream;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->eta = -1.0;
        info->bad_block = -1;
    }
    if (nrhs == 0) return 0;
    int rc = ensure_workspace(F, nrhs);
    if (rc) return rc;
    if ((rc = first(s))) return rc;
    if (F->opts.prec == PF_FP64) {
        if (info) {
            if (F->opts.flags & PF_FLAG_ETA) {
                double eta;
                if ((rc = compute_eta(F, nrhs, f, ldf, x, ldx, nullptr, n, s, &eta))) return rc;
                info->eta = eta;
            }
            if (hipStreamSynchronize(s) != hipSuccess) return PF_EHIP;
            read_status(F, info);
            return info->status;
        }
        return 0;
    }
    // FP32 bulk + FP64 refinement: x0 = solve32(f); r = f - A x; d = solve32(r); x += d
    double eta = INFINITY, prev = INFINITY;
    int iters = 0, slow = 0, status = PF_OK;
    for (;;) {
        if ((rc = compute_eta(F, nrhs, f, ldf, x, ldx, F->wsR, n, s, &eta))) return rc;
        if (eta <= F->opts.tol) break;
        // a non-finite residual (a zero pivot's infinities, say) no step mends
        if (iters >= F->opts.max_refine || !std::isfinite(eta)) { status = PF_ENOCONV; break; }
        slow = (eta > 0.5 * prev) ? slow + 1 : 0;
        if (slow >= 2) { status = PF_ENOCONV; break; }
        prev = eta;
        if ((rc = run_solve(F, nrhs, F->wsR, n, F->wsD, n, s))) return rc;
        if (launch_axpy(n, nrhs, F->wsD, n, x, ldx, s) != hipSuccess) return PF_EHIP;
        ++iters;
    }
    pf_info tmp{};
    read_status(F, &tmp);
    if (tmp.status != PF_OK) status = tmp.status;
    if (info) {
        *info = tmp;
        info->status = status;
        info->refine_iters = iters;
        info->eta = eta;
    }
    return status;
}

}  // namespace

extern "C" {

int pf_solve(pf_factor_t F, int32_t nrhs, const double *f, int64_t ldf, double *x, int64_t ldx,
             void *stream, pf_info *info)
{
    return solve_call(F, nrhs, f, ldf, x, ldx, stream, info, [&](hipStream_t s) {
        if (F->factors_stale) {   // the last factor-and-solve left no factors behind
            if (launch_factor_levels(F, s) != hipSuccess) return (int)PF_EHIP;
            F->factors_stale = false;
        }
        return run_solve(F, nrhs, f, ldf, x, ldx, s);
    });
}

int pf_factor_solve(pf_factor_t F, int32_t nrhs, const double *f, int64_t ldf, double *x,
                    int64_t ldx, void *stream, pf_info *info)
{
    if (F && nrhs == 0) {
        if (info) {
            std::memset(info, 0, sizeof *info);
            info->eta = -1.0;
            info->bad_block = -1;
        }
        return pf_refactor(F, stream);
    }
    return solve_call(F, nrhs, f, ldf, x, ldx, stream, info, [&](hipStream_t s) {
        if (F->tri_cr && nrhs == 1) return run_tri_cr(F, f, x, s);
        if (fused_ok(F, nrhs)) return run_factor_solve(F, nrhs, f, ldf, x, ldx, s);
        if (launch_factor_levels(F, s) != hipSuccess) return (int)PF_EHIP;
        return run_solve(F, nrhs, f, ldf, x, ldx, s);
    });
}

void pf_destroy(pf_factor_t F)
{
    if (!F) return;
    free_list(F, F->ws_allocs);
    free_list(F, F->allocs);
    hipStreamSynchronize(F->stream);
    pf::destroy_async(F);
}

}  // extern "C"

namespace pf {

// Release a handle whose device work is known to be complete, or whose frees
// may stay queued on its stream (stream-ordered, no host synchronization).
void destroy_async(pf_factor_s *F)
{
    if (!F) return;
    free_list(F, F->ws_allocs);
    free_list(F, F->allocs);
    for (auto *list : {&F->prof_fac, &F->prof_sol})
        for (auto &sl : *list) {
            if (sl.a) hipEventDestroy(sl.a);
            if (sl.b) hipEventDestroy(sl.b);
        }
    if (F->arena) arena_release(F->arena, F->stream);
    delete F;
}

// A new handle for A, factored and its right-hand sides solved on stream s
// in one pass per level where possible; nothing waits on the host.
int factor_new_solve(const pf_matrix *A, const pf_opts *opts, hipStream_t s, int nrhs,
                     const double *f, int64_t ldf, double *x, int64_t ldx, pf_factor_s **out,
                     const Allocator *al, double *setup_ms)
{
    *out = nullptr;
    int rc = check_matrix(A);
    if (rc) return rc;
    const pf_opts o = resolve_opts(opts);
    if ((rc = check_opts(A, o))) return rc;
    pf_factor_s *F = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    rc = factor_setup_private(A, o, s, std::max(nrhs, 1), &F, al);
    if (setup_ms)
        *setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                        .count();
    if (rc) return rc;
    if ((rc = ensure_workspace(F, std::max(nrhs, 1)))) {
        destroy_async(F);
        return rc;
    }
    if (launch_fill_u64((unsigned long long *)F->d_zero, kZeroBytes / 8, 0ull, s) != hipSuccess) {
        destroy_async(F);
        return PF_EHIP;
    }
    if (nrhs > 0 && fused_ok(F, nrhs)) rc = run_factor_solve(F, nrhs, f, ldf, x, ldx, s);
    else {
        rc = launch_factor_levels(F, s) == hipSuccess ? 0 : PF_EHIP;
        if (!rc && nrhs > 0) rc = run_solve(F, nrhs, f, ldf, x, ldx, s);
    }
    if (rc) {
        destroy_async(F);
        return rc;
    }
    *out = F;
    return 0;
}

void note_hip_error(hipError_t e) { g_last_hip = (int)e; }

// Refinement steps for a caller that must not wait (the request scheduler):
// the same kernels, in the same order, as the refinement loop of solve_call.
int ir_queue_residual(pf_factor_s *F, int nrhs, const double *f, int64_t ldf, const double *x,
                      int64_t ldx, hipStream_t s, unsigned long long *host)
{
    const int64_t n = F->nb * F->m;
    return queue_residual_norms(F, nrhs, f, ldf, x, ldx, F->wsR, n, s, host);
}
int ir_queue_correction(pf_factor_s *F, int nrhs, double *x, int64_t ldx, hipStream_t s)
{
    const int64_t n = F->nb * F->m;
    const int rc = run_solve(F, nrhs, F->wsR, n, F->wsD, n, s);
    if (rc) return rc;
    HIPCHK(launch_axpy(n, nrhs, F->wsD, n, x, ldx, s));
    return 0;
}
double ir_eta(const unsigned long long *host, int nrhs) { return eta_of(host, nrhs); }
const pf_opts &handle_opts(const pf_factor_s *F) { return F->opts; }
// a solve with stored factors and no refinement, queued on s
int solve_queued(pf_factor_s *F, int nrhs, const double *f, int64_t ldf, double *x, int64_t ldx,
                 hipStream_t s)
{
    int rc = ensure_workspace(F, nrhs);
    if (rc) return rc;
    if (F->factors_stale) {
        if (launch_factor_levels(F, s) != hipSuccess) return PF_EHIP;
        F->factors_stale = false;
    }
    return run_solve(F, nrhs, f, ldf, x, ldx, s);
}

// Factor-and-solve (pf_factor followed by pf_factor_solve, and the same
// kernels) with every device byte of the handle -- factors, reduced systems,
// status words, masked-store and zero areas, solve workspace -- carved from
// [base, base + cap): nothing is allocated on the device.  The handle itself
// is host bookkeeping, dropped before returning; the device work stays
// queued on s.  PF_ETOOBIG when the memory the plan needs exceeds cap.
int factor_solve_in(const pf_matrix *A, const pf_opts *opts, char *base, size_t cap, int nrhs,
                    const double *f, int64_t ldf, double *x, int64_t ldx, hipStream_t s,
                    pf_info *info)
{
    int rc = check_matrix(A);
    if (rc) return rc;
    const pf_opts o = resolve_opts(opts);
    if ((rc = check_opts(A, o))) return rc;
    if (o.flags & PF_FLAG_AUTOTUNE) return -2;   // tuning allocates
    if (nrhs < 0) return -3;
    const int64_t n = A->nb * A->m;
    if (nrhs > 0 && !f) return -4;
    if (ldf < n) return -5;
    if (nrhs > 0 && !x) return -6;
    if (ldx < n) return -7;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->eta = -1.0;
        info->bad_block = -1;
    }
    // the memory the plan needs: a counting pass through the same set-up
    Arena count;
    count.counting = true;
    pf_factor_s *T = nullptr;
    if ((rc = factor_setup(A, o, s, &count, nullptr, &T))) return rc;
    rc = ensure_workspace(T, std::max(nrhs, 1));
    delete T;
    if (rc) return rc;
    if (count.off + 256 > cap) return PF_ETOOBIG;
    Arena ar;
    ar.base = base;
    ar.cap = cap;
    ar.refs = 1;   // never released: the memory is not the library's to free
    pf_factor_s *F = nullptr;
    if ((rc = factor_setup(A, o, s, &ar, nullptr, &F))) return rc;
    struct Drop {
        pf_factor_s *F;
        ~Drop()
        {
            F->arena = nullptr;   // carved blocks: nothing to give back
            delete F;
        }
    } drop{F};
    if ((rc = ensure_workspace(F, std::max(nrhs, 1)))) return rc;
    HIPCHK(launch_fill_u64((unsigned long long *)F->d_zero, kZeroBytes / 8, 0ull, s));
    if (nrhs == 0) {
        HIPCHK(launch_factor_levels(F, s));
        if (!info) return 0;
        HIPCHK(hipStreamSynchronize(s));
        read_status(F, info);
        return info->status;
    }
    return solve_call(F, nrhs, f, ldf, x, ldx, (void *)s, info, [&](hipStream_t st) {
        if (F->tri_cr && nrhs == 1) return run_tri_cr(F, f, x, st);
        if (fused_ok(F, nrhs)) return run_factor_solve(F, nrhs, f, ldf, x, ldx, st);
        if (launch_factor_levels(F, st) != hipSuccess) return (int)PF_EHIP;
        return run_solve(F, nrhs, f, ldf, x, ldx, st);
    });
}

// Device status word of a handle whose work has completed (no stream wait).
int status_nosync(pf_factor_s *F, pf_info *info)
{
    std::memset(info, 0, sizeof *info);
    info->eta = -1.0;
    read_status(F, info);
    return info->status;
}

}  // namespace pf

extern "C" {

int pf_plan(const pf_matrix *A, const pf_opts *opts, int32_t max_levels, int32_t *kinds,
            int64_t *nbs, int64_t *ps)
{
    int rc = check_matrix(A);
    if (rc) return rc;
    const pf_opts o = resolve_opts(opts);
    if ((rc = check_opts(A, o))) return rc;
    const auto plan = make_plan(A->kind, A->nb, padded_block(A->m), o);
    for (int l = 0; l < (int)plan.size() && l < max_levels; ++l) {
        if (kinds) kinds[l] = plan[l].kind;
        if (nbs) nbs[l] = plan[l].nb;
        if (ps) ps[l] = plan[l].p;
    }
    return (int)plan.size();
}

int pf_factor_levels(pf_factor_t F) { return F ? (int)F->lv.size() : -1; }

int pf_factor_level(pf_factor_t F, int level, int32_t *kind, int64_t *nb, int64_t *p)
{
    if (!F) return -1;
    if (level < 0 || level >= (int)F->lv.size()) return -2;
    if (kind) *kind = F->lv[level].kind;
    if (nb) *nb = F->lv[level].nb;
    if (p) *p = F->lv[level].p;
    return 0;
}

int pf_factor_block_size(pf_factor_t F) { return F ? F->M : -1; }

int pf_factor_export_reduced(pf_factor_t F, int level, double *D, double *Lo, double *Up)
{
    if (!F) return -1;
    if (level < 0 || level + 1 >= (int)F->lv.size()) return -2;
    const Level &L = F->lv[level];
    const Level &N = F->lv[level + 1];
    const size_t bd = (size_t)F->M * F->M;
    if (hipStreamSynchronize(F->stream) != hipSuccess) return PF_EHIP;
    const size_t nD = (size_t)N.nb;
    std::vector<double> tmp(nD * bd);
    if (D) {
        if (hipMemcpy(D, L.nD, nD * bd * 8, hipMemcpyDeviceToHost) != hipSuccess) return PF_EHIP;
        if (L.nDadd) {
            if (hipMemcpy(tmp.data(), L.nDadd, nD * bd * 8, hipMemcpyDeviceToHost) != hipSuccess)
                return PF_EHIP;
            for (size_t i = 0; i < nD * bd; ++i) D[i] += tmp[i];
        }
    }
    if (Lo && hipMemcpy(Lo, L.nLo, (nD - 1) * bd * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return PF_EHIP;
    if (Up) {
        if (L.kind == PF_BTRI) {
            if (hipMemcpy(Up, L.nUp, (nD - 1) * bd * 8, hipMemcpyDeviceToHost) != hipSuccess)
                return PF_EHIP;
        } else if (hipMemcpy(Up, L.nC, bd * 8, hipMemcpyDeviceToHost) != hipSuccess) {
            return PF_EHIP;
        }
    }
    return 0;
}

int pf_band_to_btri(int64_t n, int32_t kl, int32_t ku, const double *ab, int64_t ldab,
                    double *D, double *Lo, double *Up, void *stream)
{
    if (n < 1) return -1;
    if (kl < 0) return -2;
    if (ku < 0) return -3;
    if (!ab) return -4;
    if (ldab < kl + ku + 1) return -5;
    const int m = std::max(std::max(kl, ku), 1);
    if (n % m != 0 || n / m < 2) return -1;
    if (!D) return -6;
    if (!Lo) return -7;
    if (!Up) return -8;
    return launch_band_to_btri(n, kl, ku, ab, ldab, m, D, Lo, Up, (hipStream_t)stream) ==
                   hipSuccess ? 0 : PF_EHIP;
}

struct pf_ivp_s {
    int32_t m = 0;
    int64_t p = 0, N = 0;
    hipStream_t stream = nullptr;
    double *D = nullptr, *Lo = nullptr, *C = nullptr, *f = nullptr;   // the eq. (My) system
    pf_factor_s *F = nullptr;
};

int pf_ivp_trapezoid_system(int32_t m, int64_t steps, const double *L, double h, const double *g,
                            const double *y0, double *D, double *Lo, double *C, double *f,
                            void *stream)
{
    if (m < 1) return -1;
    if (steps < 1) return -2;
    if (!L) return -3;
    if (!(h > 0.0) || !std::isfinite(h)) return -4;
    if (!g) return -5;
    if (!y0) return -6;
    if (!D) return -7;
    if (!Lo) return -8;
    if (!C) return -9;
    if (!f) return -10;
    return launch_ivp_trapezoid(m, steps, L, h, g, y0, D, Lo, C, f, (hipStream_t)stream) ==
                   hipSuccess ? 0 : PF_EHIP;
}

int pf_ivp_create(int32_t m, int64_t p, int64_t N, const pf_opts *opts, void *stream,
                  pf_ivp_t *out)
{
    if (m < 1 || m > 32) return -1;
    if (p < 1 || p > INT32_MAX) return -2;
    if (N < 2 || N > (INT64_MAX / 2) / p) return -3;
    if (!out) return -6;
    *out = nullptr;
    pf_ivp_s *I = new pf_ivp_s();
    I->m = m;
    I->p = p;
    I->N = N;
    I->stream = (hipStream_t)stream;
    const int64_t steps = p * N, nb = steps + 1;
    const size_t mm = (size_t)m * m * sizeof(double);
    hipStream_t s = I->stream;
    hipError_t e = hipMallocAsync((void **)&I->D, nb * mm, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&I->Lo, steps * mm, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&I->C, mm, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&I->f, (size_t)nb * m * sizeof(double), s);
    if (e != hipSuccess) {
        pf_ivp_destroy(I);
        return alloc_status(e);
    }
    // the coarse mesh is the partition: sub-interval i is partition i
    pf_opts o = resolve_opts(opts);
    o.partitions = (int32_t)p;
    const pf_matrix A{PF_BABD, m, nb, I->D, I->Lo, nullptr, I->C};
    int rc = check_matrix(&A);
    if (!rc) rc = check_opts(&A, o);
    if (!rc) rc = factor_setup_private(&A, o, s, 1, &I->F);
    if (!rc && launch_fill_u64((unsigned long long *)I->F->d_zero, kZeroBytes / 8, 0ull, s) != hipSuccess)
        rc = PF_EHIP;
    if (rc) {
        pf_ivp_destroy(I);
        return rc;
    }
    *out = I;
    return 0;
}

int pf_ivp_run(pf_ivp_t I, const double *L, double t0, double T, const double *g,
               const double *y0, double *y, void *stream, pf_info *info)
{
    if (!I) return -1;
    if (!L) return -2;
    if (!std::isfinite(t0) || !std::isfinite(T) || !(T > t0)) return -4;
    if (!g) return -5;
    if (!y0) return -6;
    if (!y) return -7;
    hipStream_t s = stream ? (hipStream_t)stream : I->stream;
    const int64_t steps = I->p * I->N, nb = steps + 1;
    const double h = (T - t0) / (double)steps;
    if (launch_ivp_trapezoid(I->m, steps, L, h, g, y0, I->D, I->Lo, I->C, I->f, s) != hipSuccess)
        return PF_EHIP;
    return pf_factor_solve(I->F, 1, I->f, nb * I->m, y, nb * I->m, s, info);
}

void pf_ivp_destroy(pf_ivp_t I)
{
    if (!I) return;
    if (I->F) pf_destroy(I->F);
    for (double *q : {I->D, I->Lo, I->C, I->f})
        if (q) hipFreeAsync(q, I->stream);
    hipStreamSynchronize(I->stream);
    delete I;
}

int pf_ivp_solve(int32_t m, const double *L, double t0, double T, int64_t p, int64_t N,
                 const double *g, const double *y0, double *y, const pf_opts *opts, void *stream,
                 pf_info *info)
{
    if (m < 1 || m > 32) return -1;
    if (!L) return -2;
    if (!std::isfinite(t0) || !std::isfinite(T) || !(T > t0)) return -4;
    if (p < 1 || p > INT32_MAX) return -5;
    if (N < 2 || N > (INT64_MAX / 2) / p) return -6;
    if (!g) return -7;
    if (!y0) return -8;
    if (!y) return -9;
    pf_ivp_t I = nullptr;
    int rc = pf_ivp_create(m, p, N, opts, stream, &I);
    if (rc) return rc;
    pf_info tmp;
    rc = pf_ivp_run(I, L, t0, T, g, y0, y, stream, info ? info : &tmp);
    if (!rc) rc = (info ? info : &tmp)->status;
    pf_ivp_destroy(I);
    return rc;
}

int pf_abd_to_btri(int32_t m, int64_t N, int32_t qa, const double *Ba, const double *S,
                   const double *R, const double *Bb, double *D, double *Lo, double *Up,
                   void *stream)
{
    if (m < 1) return -1;
    if (N < 1) return -2;
    if (qa < 0 || qa > m) return -3;
    if (qa > 0 && !Ba) return -4;
    if (!S) return -5;
    if (!R) return -6;
    if (qa < m && !Bb) return -7;
    if (!D) return -8;
    if (!Lo) return -9;
    if (!Up) return -10;
    return launch_abd_to_btri(m, N, qa, Ba, S, R, Bb, D, Lo, Up, (hipStream_t)stream) ==
                   hipSuccess ? 0 : PF_EHIP;
}

}  // extern "C"

// ===========================================================================
// Batches: many independent systems, one launch per (level, phase, launch
// key), the whole factor + solve sequence recorded into one HIP graph with a
// branch per block size (issue_branches).
namespace {

struct BatchLaunch {
    int phase;      // 0 factor, 1 forward sweep, 2 back substitution
    int kind, M, KC;
    bool f32, add;
    int seg;        // factor launches: segment width (0 = rows, kMapMfma = matrix cores)
    size_t work;    // first work item of this launch
    int nwg;
    int level = 0;          // recursion level of its systems
    int64_t rows = 0;       // block rows it covers (sum over its systems)
    int64_t rhs_rows = 0;   // block rows x right-hand sides (solves)
};

// Per-launch timing of a batch (pf_batch_profile): events stamped by the
// dispatches of the grouped launches.
struct BatchTimes {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<const BatchLaunch *> which;
};

// Run one grouped launch, its dispatch timed when T != NULL.
template <class Fn>
hipError_t timed_launch(BatchTimes *T, const BatchLaunch &bl, Fn fn)
{
    if (!T) return fn();
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) return hipErrorOutOfMemory;
    if (hipEventCreate(&b) != hipSuccess) {
        hipEventDestroy(a);
        return hipErrorOutOfMemory;
    }
    T->ev.push_back({a, b});
    T->which.push_back(&bl);
    LaunchTiming &t = launch_timing();
    t.start = a;
    t.stop = b;
    const hipError_t e = fn();
    t.start = t.stop = nullptr;
    return e;
}

// Device tables of one batched solve configuration (right-hand sides in,
// solutions out): kernel arguments per (system, level) and one work item
// (table entry, partition block, right-hand-side block) per workgroup.
struct SolveSet {
    SolveArgs *d_tab = nullptr;
    int4 *d_work = nullptr;
    std::vector<BatchLaunch> launches;
};

}  // namespace

struct pf_batch_s {
    int nsys = 0;
    pf_opts opts{};
    hipStream_t user = nullptr;         // the caller's stream at creation
    hipStream_t cap = nullptr;          // internal stream the graph is recorded on
    hipEvent_t ev = nullptr;
    // branches of the recorded graph: one stream and join event per block
    // size, whose launches depend on no other block size's
    std::vector<hipStream_t> lane;
    std::vector<hipEvent_t> lane_ev;
    hipEvent_t fork = nullptr;
    Arena *arena = nullptr;
    std::vector<pf_factor_s *> F;       // per system (null once handed out, or the caller's)
    std::vector<pf_factor_s *> all;     // per system, for the recorded work
    std::vector<char> ext;              // 1: the caller's existing factor, solve only
    std::vector<unsigned long long *> norms;   // per system: residual norm words
    std::vector<int32_t> nrhs;
    std::vector<const double *> f;
    std::vector<double *> x;
    std::vector<int64_t> ldf, ldx;
    unsigned long long *d_words = nullptr;   // nsys status words, nsys norm words
    LevelArgs *d_lev = nullptr;
    int4 *d_lwork = nullptr;
    std::vector<BatchLaunch> flaunch;
    SolveSet sol, corr;                  // f -> x, and residual -> correction
    // residual passes (PF_FP32_IR, PF_FLAG_ETA): one grouped launch per
    // block size with one (m in 4, 8, 16, 32), per-system launches otherwise
    struct ResGroup {
        int m = 0, nwg = 0;
        int4 *d_work = nullptr;
    };
    ResidualArgs *d_rtab = nullptr;
    std::vector<ResGroup> rgroups;
    std::vector<int> rsingle;
    // systems still refining: device mask; its pinned sources for the
    // residual pass and for the correction (two, so that the one being
    // refilled is never the source of a copy still queued)
    unsigned char *d_live = nullptr, *h_live = nullptr, *h_live2 = nullptr;
    AxpyArgs *d_atab = nullptr;          // x += d of the refinement, one launch
    int4 *d_awork = nullptr;
    int anwg = 0;
    std::vector<void *> own;             // table allocations
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

hipError_t launch_pad_matrix(pf_factor_s *F, hipStream_t s)
{
    const pf_matrix &A0 = F->A;
    hipError_t e = launch_pad_blocks(A0.m, F->M, A0.nb, A0.D, F->padD, 1.0, s);
    if (e == hipSuccess) e = launch_pad_blocks(A0.m, F->M, A0.nb - 1, A0.Lo, F->padLo, 0.0, s);
    if (e == hipSuccess && F->padUp)
        e = launch_pad_blocks(A0.m, F->M, A0.nb - 1, A0.Up, F->padUp, 0.0, s);
    if (e == hipSuccess && F->padC) e = launch_pad_blocks(A0.m, F->M, 1, A0.C, F->padC, 0.0, s);
    return e;
}

void build_factor_tables(pf_batch_s *B, std::vector<LevelArgs> &tab, std::vector<int4> &work)
{
    size_t maxL = 0;
    for (auto *F : B->all) maxL = std::max(maxL, F->lv.size());
    for (size_t l = 0; l < maxL; ++l) {
        std::map<std::tuple<int, int, int, int, int>, std::vector<int>> groups;
        for (int i = 0; i < B->nsys; ++i) {
            const pf_factor_s *F = B->all[i];
            if (l >= F->lv.size() || B->ext[i]) continue;
            const Level &L = F->lv[l];
            groups[{L.kind, F->M, L.f32 ? 1 : 0, (L.kind == PF_BTRI && L.Dadd) ? 1 : 0,
                    L.seg}].push_back(i);
        }
        for (auto &kv : groups) {
            BatchLaunch bl{0, std::get<0>(kv.first), std::get<1>(kv.first), 1,
                           std::get<2>(kv.first) != 0, std::get<3>(kv.first) != 0,
                           std::get<4>(kv.first), work.size(), 0};
            const int gpw = bl.seg == kMapMfma   ? mfma_partitions_per_wg()
                            : bl.seg == kMapMfma32 || bl.seg == kMapMfmaB16 || bl.seg == kMapMfma16 ? 1
                            : bl.seg             ? seg_partitions_per_wg(bl.M, bl.seg)
                                                 : groups_per_wg(bl.M);
            bl.level = (int)l;
            for (int i : kv.second) {
                const int entry = (int)tab.size();
                tab.push_back(level_args(B->all[i], l));
                bl.rows += B->all[i]->lv[l].nb;
                const int64_t nblk = (B->all[i]->lv[l].p + gpw - 1) / gpw;
                for (int64_t pb = 0; pb < nblk; ++pb) work.push_back(make_int4(entry, (int)pb, 0, 0));
            }
            bl.nwg = (int)(work.size() - bl.work);
            B->flaunch.push_back(bl);
        }
    }
}

// rhs/sol: per-system level-0 right-hand sides and solutions (unpadded);
// systems whose block size is padded run through their padded workspace.
void build_solve_tables(pf_batch_s *B, const std::vector<const double *> &rhs,
                        const std::vector<int64_t> &ldr, const std::vector<double *> &sol,
                        const std::vector<int64_t> &lds, SolveSet &S, std::vector<SolveArgs> &tab,
                        std::vector<int4> &work)
{
    std::vector<std::vector<SolveArgs>> args(B->nsys);
    size_t maxL = 0;
    for (int i = 0; i < B->nsys; ++i) {
        pf_factor_s *F = B->all[i];
        const bool pad = F->M != F->m;
        const int64_t ldp = F->nb * F->M;
        args[i] = solve_args(F, B->nrhs[i], pad ? F->wsPadF : rhs[i], pad ? ldp : ldr[i],
                             pad ? F->wsPadX : sol[i], pad ? ldp : lds[i]);
        maxL = std::max(maxL, F->lv.size());
    }
    auto emit = [&](int phase, size_t l) {
        // partitions per (kind, block size, precision, ADD) class of the
        // level: the launches of a class share them
        std::map<std::tuple<int, int, int, int>, int64_t> parts;
        auto cls = [&](int i) {
            const Level &L = B->all[i]->lv[l];
            const int add = (phase == 1 && L.kind == PF_BTRI && args[i][l].Fadd) ? 1 : 0;
            return std::make_tuple(L.kind, B->all[i]->M, L.f32 ? 1 : 0, add);
        };
        for (int i = 0; i < B->nsys; ++i)
            if (l < B->all[i]->lv.size() && B->nrhs[i] > 0) parts[cls(i)] += B->all[i]->lv[l].p;
        std::map<std::tuple<int, int, int, int, int>, std::vector<int>> groups;
        for (int i = 0; i < B->nsys; ++i) {
            const pf_factor_s *F = B->all[i];
            if (l >= F->lv.size() || B->nrhs[i] == 0) continue;
            const Level &L = F->lv[l];
            const auto c = cls(i);
            groups[{L.kind, F->M, L.f32 ? 1 : 0, std::get<3>(c),
                    solve_cols(F->M, L.f32, L.kind == PF_BTRI && !std::get<3>(c), B->nrhs[i], parts[c])}]
                .push_back(i);
        }
        for (auto &kv : groups) {
            BatchLaunch bl{phase, std::get<0>(kv.first), std::get<1>(kv.first),
                           std::get<4>(kv.first), std::get<2>(kv.first) != 0,
                           std::get<3>(kv.first) != 0, 0, work.size(), 0};
            const int gpw = solve_groups_per_wg(bl.M, bl.f32);
            bl.level = (int)l;
            for (int i : kv.second) {
                const int entry = (int)tab.size();
                tab.push_back(args[i][l]);
                bl.rows += B->all[i]->lv[l].nb;
                bl.rhs_rows += B->all[i]->lv[l].nb * B->nrhs[i];
                const int64_t nblk = (B->all[i]->lv[l].p + gpw - 1) / gpw;
                const int ncb = (B->nrhs[i] + bl.KC - 1) / bl.KC;
                for (int cb = 0; cb < ncb; ++cb)
                    for (int64_t pb = 0; pb < nblk; ++pb)
                        work.push_back(make_int4(entry, (int)pb, cb, 0));
            }
            bl.nwg = (int)(work.size() - bl.work);
            S.launches.push_back(bl);
        }
    };
    for (size_t l = 0; l < maxL; ++l) emit(1, l);
    for (size_t l = maxL; l-- > 0;) emit(2, l);
}

// Status words cleared and padded copies of the matrices made: what every
// factor launch of the batch depends on.
hipError_t factor_prologue(pf_batch_s *B, hipStream_t s)
{
    hipError_t e = launch_fill_u64(B->d_words, B->nsys, ~0ull, s);
    if (e == hipSuccess) e = launch_fill_u64(B->d_words + B->nsys, B->nsys, 0ull, s);
    for (int i = 0; i < B->nsys; ++i)
        if (e == hipSuccess && !B->ext[i] && B->all[i]->M != B->all[i]->m)
            e = launch_pad_matrix(B->all[i], s);
    return e;
}

hipError_t factor_launch(pf_batch_s *B, const BatchLaunch &bl, hipStream_t s, BatchTimes *T)
{
    return timed_launch(T, bl, [&] { return
              bl.seg == kMapMfma ? launch_mfma_factor_batch(B->d_lev, B->d_lwork + bl.work, bl.nwg, s)
                : bl.seg == kMapMfma32
                    ? launch_mfma32_factor_batch(bl.add, bl.f32, B->d_lev, B->d_lwork + bl.work, bl.nwg, s)
                : bl.seg == kMapMfmaB16
                    ? launch_mfma_babd16_factor_batch(bl.f32, B->d_lev, B->d_lwork + bl.work, bl.nwg, s)
                : bl.seg == kMapMfma16
                    ? launch_mfma16_factor_batch(bl.add, bl.f32, B->d_lev, B->d_lwork + bl.work, bl.nwg, s)
                : bl.seg ? launch_seg_factor_batch(bl.kind, bl.M, bl.seg, bl.f32, bl.add, B->d_lev,
                                                   B->d_lwork + bl.work, bl.nwg, s)
                         : launch_factor_batch(bl.kind, bl.M, bl.f32, bl.add, B->d_lev,
                                               B->d_lwork + bl.work, bl.nwg, s); });
}

hipError_t issue_factor(pf_batch_s *B, hipStream_t s, BatchTimes *T = nullptr)
{
    hipError_t e = factor_prologue(B, s);
    for (const auto &bl : B->flaunch)
        if (e == hipSuccess) e = factor_launch(B, bl, s, T);
    return e;
}

// right-hand sides of systems with a padded block size into their padded
// workspace (before the solve launches), solutions back (after)
hipError_t solve_pad(pf_batch_s *B, bool corr, bool in, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int i = 0; i < B->nsys && e == hipSuccess; ++i) {
        pf_factor_s *F = B->all[i];
        if (F->M == F->m || B->nrhs[i] == 0) continue;
        const int64_t n = F->nb * F->m;
        if (in)
            e = launch_pad_rhs(F->m, F->M, F->nb, B->nrhs[i], corr ? F->wsR : B->f[i],
                               corr ? n : B->ldf[i], F->wsPadF, F->nb * F->M, true, s);
        else
            e = launch_pad_rhs(F->m, F->M, F->nb, B->nrhs[i], F->wsPadX, F->nb * F->M,
                               corr ? F->wsD : B->x[i], corr ? n : B->ldx[i], false, s);
    }
    return e;
}

hipError_t solve_launch(const SolveSet &S, const BatchLaunch &bl, hipStream_t s, BatchTimes *T)
{
    return timed_launch(T, bl, [&] {
        return launch_solve_batch(bl.kind, bl.phase == 1, bl.M, bl.f32, bl.add, bl.KC, S.d_tab,
                                  S.d_work + bl.work, bl.nwg, s);
    });
}

hipError_t issue_solve(pf_batch_s *B, const SolveSet &S, bool corr, hipStream_t s,
                       BatchTimes *T = nullptr)
{
    hipError_t e = solve_pad(B, corr, true, s);
    for (const auto &bl : S.launches)
        if (e == hipSuccess) e = solve_launch(S, bl, s, T);
    if (e == hipSuccess) e = solve_pad(B, corr, false, s);
    return e;
}

// The recorded graph: the prologues on s, then the systems of each block
// size on a branch of their own -- their factor launches level by level,
// then their solve launches -- the branches joined back into s before the
// solutions are unpadded.  Launch for launch the work of issue_factor and
// issue_solve; the block sizes only no longer wait for each other.  (Not
// the kinds: the last level of a bidiagonal-plus-corner system is block
// tridiagonal, in the launches of that kind.)
// (With factor == false: the solve set S alone, as the refinement's
// correction solves are issued, on the same branch streams, eagerly.)
hipError_t issue_branches(pf_batch_s *B, hipStream_t s, bool factor, const SolveSet &S, bool corr)
{
    hipError_t e = factor ? factor_prologue(B, s) : hipSuccess;
    if (e == hipSuccess) e = solve_pad(B, corr, true, s);
    if (e == hipSuccess) e = hipEventRecord(B->fork, s);
    // largest block size first: its branch is the longest
    std::map<int, size_t, std::greater<int>> cls;
    if (factor)
        for (const auto &bl : B->flaunch) cls.emplace(bl.M, cls.size());
    for (const auto &bl : S.launches) cls.emplace(bl.M, cls.size());
    for (const auto &c : cls) {
        if (e != hipSuccess) break;
        if (c.second >= B->lane.size()) return hipErrorInvalidValue;
        hipStream_t ls = B->lane[c.second];
        e = hipStreamWaitEvent(ls, B->fork, 0);
        if (factor)
            for (const auto &bl : B->flaunch)
                if (e == hipSuccess && bl.M == c.first) e = factor_launch(B, bl, ls, nullptr);
        for (const auto &bl : S.launches)
            if (e == hipSuccess && bl.M == c.first) e = solve_launch(S, bl, ls, nullptr);
        if (e == hipSuccess) e = hipEventRecord(B->lane_ev[c.second], ls);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, B->lane_ev[c.second], 0);
    }
    if (e == hipSuccess) e = solve_pad(B, corr, false, s);
    return e;
}

template <class T>
hipError_t upload(pf_batch_s *B, const std::vector<T> &v, T **d)
{
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return e;
    B->own.push_back(p);
    *d = (T *)p;
    return v.empty() ? hipSuccess : hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

void batch_free(pf_batch_s *B)
{
    if (B->cap) hipStreamSynchronize(B->cap);
    if (B->exec) hipGraphExecDestroy(B->exec);
    if (B->graph) hipGraphDestroy(B->graph);
    for (hipStream_t ls : B->lane) hipStreamDestroy(ls);
    for (hipEvent_t le : B->lane_ev) hipEventDestroy(le);
    if (B->fork) hipEventDestroy(B->fork);
    for (auto *F : B->F)
        if (F) pf_destroy(F);
    for (void *p : B->own) hipFree(p);
    if (B->h_live) hipHostFree(B->h_live);
    if (B->h_live2) hipHostFree(B->h_live2);
    if (B->arena) arena_release(B->arena, B->cap ? B->cap : B->user);
    if (B->ev) hipEventDestroy(B->ev);
    if (B->cap) hipStreamDestroy(B->cap);
    delete B;
}

// FP64 refinement of every system of the batch (PF_FP32_IR): residuals and
// norms for all systems, one synchronization, then one batched correction
// solve for all systems, until every eta <= tol or a system stagnates.
int batch_refine(pf_batch_s *B, hipStream_t s, bool refine, std::vector<double> &eta,
                 std::vector<int> &iters, std::vector<int> &status)
{
    const int ns = B->nsys;
    eta.assign(ns, INFINITY);
    iters.assign(ns, 0);
    status.assign(ns, PF_OK);
    std::vector<double> prev(ns, INFINITY);
    std::vector<int> slow(ns, 0), done(ns, 0);
    // words: ns status, ns ||A||, then 3 * max(nrhs, 1) norms per system
    size_t slots = 0;
    for (int i = 0; i < ns; ++i) slots += 3 * (size_t)std::max(B->nrhs[i], 1);
    std::vector<unsigned long long> h(2 * (size_t)ns + slots);
    // ||A||_inf (zeroed with the status words when the graph starts) comes
    // with the first residual of each system
    for (bool first = true;; first = false) {
        HIPCHK(launch_fill_u64(B->d_words + 2 * ns, (int64_t)slots, 0ull, s));
        for (int i = 0; i < ns; ++i) B->h_live[i] = (!done[i] && B->nrhs[i] > 0) ? 1 : 0;
        // pinned source: queued, not waited on (the sweep's synchronization
        // below comes before the next change of h_live)
        HIPCHK(hipMemcpyAsync(B->d_live, B->h_live, ns, hipMemcpyHostToDevice, s));
        for (const auto &G : B->rgroups)
            HIPCHK(launch_residual_batch(G.m, B->d_rtab, G.d_work, G.nwg, B->d_live, first, refine, s));
        for (int i : B->rsingle) {
            pf_factor_s *F = B->all[i];
            const pf_matrix &A = F->A;
            const int64_t n = A.nb * A.m;
            if (!B->h_live[i]) continue;
            HIPCHK(launch_residual(A.kind, A.m, A.nb, A.D, A.Lo, A.Up, A.C, B->nrhs[i], B->f[i],
                                   B->ldf[i], B->x[i], B->ldx[i], refine ? F->wsR : nullptr, n,
                                   B->norms[i], first ? B->d_words + ns + i : nullptr, s));
        }
        HIPCHK(hipMemcpyAsync(h.data(), B->d_words, h.size() * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        bool all = true;
        size_t off = 2 * (size_t)ns;
        for (int i = 0; i < ns; ++i) {
            const size_t base = off;
            off += 3 * (size_t)std::max(B->nrhs[i], 1);
            if (done[i]) continue;
            const double na = bits_to_double(h[ns + i]);
            double w = 0.0;
            for (int c = 0; c < B->nrhs[i]; ++c) {
                const double nr = bits_to_double(h[base + 3 * c]),
                             nx = bits_to_double(h[base + 3 * c + 1]),
                             nf = bits_to_double(h[base + 3 * c + 2]);
                const double den = na * nx + nf;
                double e = den > 0 ? nr / den : (nr > 0 ? INFINITY : 0.0);
                if (std::isnan(e)) e = INFINITY;
                w = std::max(w, e);
            }
            eta[i] = w;
            if (!refine) continue;   // eta only (FP64 with PF_FLAG_ETA)
            if (w <= B->opts.tol) { done[i] = 1; continue; }
            if (iters[i] >= B->opts.max_refine || !std::isfinite(w)) {
                done[i] = 1;
                status[i] = PF_ENOCONV;
                continue;
            }
            slow[i] = (w > 0.5 * prev[i]) ? slow[i] + 1 : 0;
            if (slow[i] >= 2) { done[i] = 1; status[i] = PF_ENOCONV; continue; }
            prev[i] = w;
            all = false;
        }
        if (all || !refine) break;
        HIPCHK(issue_branches(B, s, false, B->corr, true));
        for (int i = 0; i < ns; ++i) {
            B->h_live2[i] = (!done[i] && B->nrhs[i] > 0) ? 1 : 0;
            if (!done[i]) ++iters[i];
        }
        HIPCHK(hipMemcpyAsync(B->d_live, B->h_live2, ns, hipMemcpyHostToDevice, s));
        HIPCHK(launch_axpy_batch(B->d_atab, B->d_awork, B->anwg, B->d_live, s));
    }
    return 0;
}

// A batch; existing (may be NULL): per system the caller's factor of A[i]
// (solved with, not factored) or NULL (factored by the batch).  Argument
// errors are numbered as pf_solve_batch numbers them (existing = 10).
// Finest-level chain length in a batch.  One grouped launch runs the
// partitions of every system with the same kind and block size, so a batch
// has parallelism to spare where one system of the same shape does not: each
// such group takes spare_chain over the block rows of all its systems (block
// size 32, 139 systems, 1.38 M block rows: 63.8 ms of kernel time with 4
// blocks per partition, 57.0 with 32, 57.0 with 64, 57.9 with 128; on the
// 512-system batch the rule picks 64 for every block size, within 1 % of the
// measured best, 32 or 64, of each).  Systems whose chain length is fixed --
// by the caller, the autotuner or a partition count -- keep it, and so do
// scalar systems.
void batch_chain_lengths(int32_t nsys, const pf_matrix *A, const pf_opts &o,
                         pf_factor_s *const *existing, std::vector<pf_opts> &os)
{
    if (o.block_rows > 0 || o.partitions > 0) return;
    auto open = [&](int i) {
        return !(existing && existing[i]) && os[i].block_rows == 0 && os[i].partitions == 0 &&
               padded_block(A[i].m) > 1;
    };
    std::map<std::pair<int, int>, int64_t> rows;   // (kind, block size) -> block rows
    for (int i = 0; i < nsys; ++i)
        if (open(i)) rows[{A[i].kind, padded_block(A[i].m)}] += A[i].nb;
    for (const auto &g : rows) {
        const int kind = g.first.first, M = g.first.second;
        const int L = spare_chain(target_rows(kind, M, o.prec == PF_FP32_IR, 0, o), g.second);
        for (int i = 0; i < nsys; ++i)
            if (open(i) && A[i].kind == kind && padded_block(A[i].m) == M) os[i].block_rows = L;
    }
}

int batch_create(int32_t nsys, const pf_matrix *A, const pf_opts *opts, const int32_t *nrhs,
                 const double *const *f, const int64_t *ldf, double *const *x,
                 const int64_t *ldx, void *stream, pf_factor_s *const *existing, pf_batch_t *out)
{
    *out = nullptr;
    if (nsys < 1) return -1;
    if (!A) return -2;
    const pf_opts o = resolve_opts(opts);
    if (!nrhs || !f || !ldf || !x || !ldx) return -4;
    for (int i = 0; i < nsys; ++i) {
        int rc = check_matrix(&A[i]);
        if (rc) return rc < 0 ? -2 : rc;
        if ((rc = check_opts(&A[i], o))) return -3;
        const int64_t n = A[i].nb * A[i].m;
        if (nrhs[i] < 0 || (nrhs[i] > 0 && (!f[i] || !x[i])) || ldf[i] < n || ldx[i] < n) return -4;
        const pf_factor_s *E = existing ? existing[i] : nullptr;
        if (E && (E->A.kind != A[i].kind || E->m != A[i].m || E->nb != A[i].nb ||
                  E->opts.prec != o.prec))
            return -10;
    }
    hipStream_t us = (hipStream_t)stream;
    // per-system launch shapes (the autotuner's, when asked for)
    std::vector<pf_opts> os(nsys, o);
    if (o.flags & PF_FLAG_AUTOTUNE)
        for (int i = 0; i < nsys; ++i) {
            if (existing && existing[i]) continue;
            pf_opts t{};
            const int rc = tuned_opts(&A[i], o, std::max(nrhs[i], 1), us, &t);
            if (rc) return rc;
            os[i] = resolve_opts(&t);
        }
    batch_chain_lengths(nsys, A, o, existing, os);
    pf_batch_s *B = new pf_batch_s();
    B->nsys = nsys;
    B->opts = o;
    B->user = us;
    B->nrhs.assign(nrhs, nrhs + nsys);
    B->ext.assign(nsys, 0);
    if (existing)
        for (int i = 0; i < nsys; ++i) B->ext[i] = existing[i] != nullptr;
    B->f.assign(f, f + nsys);
    B->x.assign(x, x + nsys);
    B->ldf.assign(ldf, ldf + nsys);
    B->ldx.assign(ldx, ldx + nsys);
    auto fail = [&](int code) {
        batch_free(B);
        return code;
    };
    if (hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess) return fail(PF_EHIP);
    if (hipEventCreateWithFlags(&B->ev, hipEventDisableTiming) != hipSuccess) return fail(PF_EHIP);

    // sizes: a counting pass through the same setup code
    Arena count;
    count.counting = true;
    size_t total_rhs = 0;
    for (int i = 0; i < nsys; ++i) total_rhs += (size_t)std::max(nrhs[i], 1);
    const size_t words = (2 * (size_t)nsys + 3 * total_rhs) * sizeof(unsigned long long);
    void *fake = (void *)(uintptr_t)4096;
    for (int i = 0; i < nsys; ++i) {
        if (B->ext[i]) continue;
        pf_factor_s *F = nullptr;
        if (factor_setup(&A[i], os[i], us, &count, fake, &F)) return fail(PF_ENOMEM);
        ensure_workspace(F, std::max(nrhs[i], 1));
        delete F;
    }
    B->arena = new Arena();
    B->arena->refs = 1;
    B->arena->cap = count.off + words + kDumpBytes + kZeroBytes + 4096;
    B->arena->al = g_allocator;
    {
        const hipError_t e = dev_alloc(B->arena->al, (void **)&B->arena->base, B->arena->cap, us);
        if (e != hipSuccess) return fail(alloc_status(e));
    }
    Arena &ar = *B->arena;
    B->d_words = (unsigned long long *)ar.base;
    ar.off = words;
    void *scratch = ar.base + ((ar.off + 255) & ~(size_t)255);
    ar.off = ((ar.off + 255) & ~(size_t)255) + kDumpBytes + kZeroBytes;
    unsigned long long *norms = B->d_words + 2 * nsys;
    B->F.assign(nsys, nullptr);
    B->all.assign(nsys, nullptr);
    B->norms.assign(nsys, nullptr);
    for (int i = 0; i < nsys; ++i) {
        B->norms[i] = norms;
        norms += 3 * (size_t)std::max(nrhs[i], 1);
        if (B->ext[i]) {
            // the caller's handle: its own memory, its workspace grown if needed
            pf_factor_s *F = existing[i];
            const int rc = ensure_workspace(F, std::max(nrhs[i], 1));
            if (rc) return fail(rc);
            if (F->stream != us && hipStreamSynchronize(F->stream) != hipSuccess) return fail(PF_EHIP);
            B->all[i] = F;
            continue;
        }
        pf_factor_s *F = nullptr;
        int rc = factor_setup(&A[i], os[i], us, B->arena, scratch, &F);
        if (rc) return fail(rc);
        ++ar.refs;
        B->F[i] = F;
        // grouped launches run the segment kernels (same arithmetic)
        for (Level &L : F->lv)
            if (L.seg == kMapTri) L.seg = 1;
        if ((rc = ensure_workspace(F, std::max(nrhs[i], 1)))) return fail(rc);
        // status, ||A|| and per-column norm words of all systems are
        // contiguous: one fill, one read-back per refinement sweep
        F->d_status = B->d_words + i;
        F->d_norm = B->d_words + nsys + i;
        F->d_norms = B->norms[i];
        B->all[i] = F;
    }
    if (launch_fill_u64((unsigned long long *)((char *)scratch + kDumpBytes), kZeroBytes / 8, 0ull,
                        us) != hipSuccess)
        return fail(PF_EHIP);

    std::vector<LevelArgs> ltab;
    std::vector<int4> lwork;
    build_factor_tables(B, ltab, lwork);
    std::vector<SolveArgs> stab, ctab;
    std::vector<int4> swork, cwork;
    build_solve_tables(B, B->f, B->ldf, B->x, B->ldx, B->sol, stab, swork);
    if (o.prec == PF_FP32_IR) {
        std::vector<const double *> r(nsys);
        std::vector<double *> d(nsys);
        std::vector<int64_t> ld(nsys);
        for (int i = 0; i < nsys; ++i) {
            r[i] = B->all[i]->wsR;
            d[i] = B->all[i]->wsD;
            ld[i] = B->all[i]->nb * B->all[i]->m;
        }
        build_solve_tables(B, r, ld, d, ld, B->corr, ctab, cwork);
    }
    if (upload(B, ltab, &B->d_lev) || upload(B, lwork, &B->d_lwork) ||
        upload(B, stab, &B->sol.d_tab) || upload(B, swork, &B->sol.d_work))
        return fail(PF_EHIP);
    if (o.prec == PF_FP32_IR &&
        (upload(B, ctab, &B->corr.d_tab) || upload(B, cwork, &B->corr.d_work)))
        return fail(PF_EHIP);
    if (o.prec == PF_FP32_IR || (o.flags & PF_FLAG_ETA)) {
        // residual tables: per system its operands; per block size with a
        // grouped launch, work units of a few runs of steps
        std::vector<ResidualArgs> rtab(nsys);
        std::map<int, std::vector<int4>> rwork;
        for (int i = 0; i < nsys; ++i) {
            pf_factor_s *F = B->all[i];
            const pf_matrix &A = F->A;
            const int64_t n = A.nb * A.m;
            rtab[i] = ResidualArgs{A.kind, A.m, A.nb, A.D, A.Lo, A.Up, A.C, nrhs[i], B->f[i],
                                   B->ldf[i], B->x[i], B->ldx[i], F->wsR, n, B->norms[i],
                                   B->d_words + nsys + i};
            if (!residual_batched(A.m)) {
                B->rsingle.push_back(i);
                continue;
            }
            const int64_t steps = (n + residual_step_rows(A.m) - 1) / residual_step_rows(A.m);
            const int per = residual_item_steps();
            if (steps > INT32_MAX - per) {
                B->rsingle.push_back(i);
                continue;
            }
            const int chunks = (nrhs[i] + 63) / 64;
            auto &w = rwork[A.m];
            for (int c = 0; c < chunks; ++c)
                for (int64_t t = 0; t < steps; t += per)
                    w.push_back(int4{i, (int)t, (int)std::min<int64_t>(t + per, steps), c});
        }
        if (upload(B, rtab, &B->d_rtab)) return fail(PF_EHIP);
        for (auto &kv : rwork) {
            pf_batch_s::ResGroup G;
            G.m = kv.first;
            G.nwg = (int)kv.second.size();
            if (upload(B, kv.second, &G.d_work)) return fail(PF_EHIP);
            B->rgroups.push_back(G);
        }
        std::vector<unsigned char> live(nsys, 1);
        if (upload(B, live, &B->d_live)) return fail(PF_EHIP);
        if (hipHostMalloc((void **)&B->h_live, nsys, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&B->h_live2, nsys, hipHostMallocDefault) != hipSuccess)
            return fail(PF_EHIP);
        if (o.prec == PF_FP32_IR) {
            std::vector<AxpyArgs> atab(nsys);
            std::vector<int4> awork;
            for (int i = 0; i < nsys; ++i) {
                pf_factor_s *F = B->all[i];
                const int64_t n = F->nb * F->m;
                atab[i] = AxpyArgs{B->x[i], F->wsD, n, B->ldx[i], n, nrhs[i]};
                const int64_t units = (n * nrhs[i] + kAxpyUnit - 1) / kAxpyUnit;
                for (int64_t u = 0; u < units; u += 4)
                    awork.push_back(int4{i, (int)u, (int)std::min<int64_t>(u + 4, units), 0});
            }
            if (upload(B, atab, &B->d_atab) || upload(B, awork, &B->d_awork)) return fail(PF_EHIP);
            B->anwg = (int)awork.size();
        }
    }
    if (hipStreamSynchronize(us) != hipSuccess) return fail(PF_EHIP);

    // record factor + solve once, one branch per block size;
    // pf_batch_run replays it
    {
        std::set<int> cls;
        for (const auto &bl : B->flaunch) cls.insert(bl.M);
        for (const auto &bl : B->sol.launches) cls.insert(bl.M);
        if (hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) != hipSuccess) return fail(PF_EHIP);
        for (size_t c = 0; c < cls.size(); ++c) {
            hipStream_t ls = nullptr;
            hipEvent_t le = nullptr;
            if (hipStreamCreateWithFlags(&ls, hipStreamNonBlocking) != hipSuccess) return fail(PF_EHIP);
            B->lane.push_back(ls);
            if (hipEventCreateWithFlags(&le, hipEventDisableTiming) != hipSuccess) return fail(PF_EHIP);
            B->lane_ev.push_back(le);
        }
    }
    if (hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(PF_EHIP);
    hipError_t e = issue_branches(B, B->cap, true, B->sol, false);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(B->cap, &g);
    B->graph = g;
    if (e != hipSuccess || e2 != hipSuccess || !g) return fail(PF_EHIP);
    if (hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0) != hipSuccess)
        return fail(PF_EHIP);
    *out = B;
    return 0;
}

}  // namespace

extern "C" {

int pf_batch_create(int32_t nsys, const pf_matrix *A, const pf_opts *opts, const int32_t *nrhs,
                    const double *const *f, const int64_t *ldf, double *const *x,
                    const int64_t *ldx, void *stream, pf_batch_t *out)
{
    if (!out) return -10;
    return batch_create(nsys, A, opts, nrhs, f, ldf, x, ldx, stream, nullptr, out);
}

int pf_batch_run(pf_batch_t B, void *stream, pf_info *info)
{
    if (!B) return -1;
    hipStream_t us = (hipStream_t)stream;
    if (hipEventRecord(B->ev, us) != hipSuccess) return PF_EHIP;
    if (hipStreamWaitEvent(B->cap, B->ev, 0) != hipSuccess) return PF_EHIP;
    if (hipGraphLaunch(B->exec, B->cap) != hipSuccess) return PF_EHIP;
    std::vector<double> eta;
    std::vector<int> iters, st;
    int worst = 0;
    if (B->opts.prec == PF_FP32_IR || (B->opts.flags & PF_FLAG_ETA)) {
        const int rc = batch_refine(B, B->cap, B->opts.prec == PF_FP32_IR, eta, iters, st);
        if (rc) return rc;
    }
    if (hipEventRecord(B->ev, B->cap) != hipSuccess) return PF_EHIP;
    if (hipStreamWaitEvent(us, B->ev, 0) != hipSuccess) return PF_EHIP;
    if (info || B->opts.prec == PF_FP32_IR) {
        if (hipStreamSynchronize(B->cap) != hipSuccess) return PF_EHIP;
        std::vector<unsigned long long> w(B->nsys);
        if (hipMemcpy(w.data(), B->d_words, B->nsys * sizeof(unsigned long long),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return PF_EHIP;
        for (int i = 0; i < B->nsys; ++i) {
            pf_info inf{};
            inf.eta = -1.0;
            inf.bad_block = -1;
            if (w[i] != ~0ull) {
                inf.status = PF_ESINGULAR;
                inf.bad_level = (int32_t)(w[i] >> 40);
                inf.bad_block = (int64_t)(w[i] & ((1ull << 40) - 1));
            }
            if (!eta.empty()) {
                inf.eta = eta[i];
                inf.refine_iters = iters[i];
                if (inf.status == PF_OK) inf.status = st[i];
            }
            if (inf.status && !worst) worst = inf.status;
            if (info) info[i] = inf;
        }
    }
    return worst;
}

int pf_batch_profile(pf_batch_t B, void *stream, int32_t max, pf_launch_info *out,
                     int32_t *count)
{
    if (!B) return -1;
    if (max < 0 || (max > 0 && !out)) return -3;
    if (!count) return -5;
    *count = 0;
    hipStream_t us = (hipStream_t)stream;
    HIPCHK(hipEventRecord(B->ev, us));
    HIPCHK(hipStreamWaitEvent(B->cap, B->ev, 0));
    BatchTimes T;
    hipError_t e = issue_factor(B, B->cap, &T);
    if (e == hipSuccess) e = issue_solve(B, B->sol, false, B->cap, &T);
    const hipError_t es = hipStreamSynchronize(B->cap);
    int n = 0;
    for (size_t i = 0; i < T.ev.size(); ++i, ++n) {
        float ms = -1.f;
        if (e == hipSuccess && es == hipSuccess &&
            hipEventElapsedTime(&ms, T.ev[i].first, T.ev[i].second) != hipSuccess)
            ms = -1.f;
        hipEventDestroy(T.ev[i].first);
        hipEventDestroy(T.ev[i].second);
        if (n >= max) continue;
        const BatchLaunch &bl = *T.which[i];
        pf_launch_info &o = out[n];
        o.phase = bl.phase;
        o.level = bl.level;
        o.kind = bl.kind;
        o.m = bl.M;
        o.f32 = bl.f32 ? 1 : 0;
        o.mapping = bl.phase == 0 ? bl.seg : 0;
        o.rows = bl.rows;
        o.rhs_rows = bl.rhs_rows;
        o.workgroups = bl.nwg;
        o.ms = ms;
    }
    *count = n;
    if (e != hipSuccess || es != hipSuccess) {
        g_last_hip = (int)(e != hipSuccess ? e : es);
        return PF_EHIP;
    }
    return 0;
}

int pf_batch_factor(pf_batch_t B, int32_t i, pf_factor_t *out)
{
    if (!B) return -1;
    if (i < 0 || i >= B->nsys) return -2;
    if (!out) return -3;
    *out = B->F[i];
    if (!B->F[i]) return -2;      // already handed out
    B->F[i] = nullptr;            // the handle now owns its share of the arena
    return 0;
}

void pf_batch_destroy(pf_batch_t B)
{
    if (B) batch_free(B);
}

int pf_solve_batch(int32_t nsys, const pf_matrix *A, const pf_opts *opts, const int32_t *nrhs,
                   const double *const *f, const int64_t *ldf, double *const *x,
                   const int64_t *ldx, void *stream, pf_factor_t *factors, pf_info *info)
{
    if (nsys < 0) return -1;
    if (nsys == 0) return 0;
    pf_batch_t B = nullptr;
    int rc = batch_create(nsys, A, opts, nrhs, f, ldf, x, ldx, stream, factors, &B);
    if (rc) return rc;
    std::vector<pf_info> tmp(nsys);
    rc = pf_batch_run(B, stream, info ? info : tmp.data());
    if (factors)
        for (int i = 0; i < nsys; ++i)
            if (!B->ext[i]) pf_batch_factor(B, i, &factors[i]);
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && !rc) rc = PF_EHIP;
    pf_batch_destroy(B);
    return rc;
}

}  // extern "C"
