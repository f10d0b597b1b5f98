// Host side of the partition-method library: argument checks, the level
// plan of the recursion, device memory of a factor handle, the solve
// orchestration (forward sweeps down the levels, back substitution up) and
// FP64 iterative refinement.
#include "pf.h"
#include "pf_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

using namespace pf;

namespace {

struct Level {
    int kind = PF_BTRI;
    int64_t nb = 0, p = 1;
    bool f32 = false;
    const double *D = nullptr, *Dadd = nullptr, *Lo = nullptr, *Up = nullptr, *C = nullptr;
    void *E = nullptr, *R = nullptr, *Z = nullptr, *X = nullptr;
    double *nD = nullptr, *nDadd = nullptr, *nLo = nullptr, *nUp = nullptr, *nC = nullptr;
};

struct PlanLevel {
    int kind;
    int64_t nb, p;
};

}  // namespace

struct pf_factor_s {
    pf_matrix A{};
    pf_opts opts{};
    int m = 0, M = 0;
    int64_t nb = 0;
    hipStream_t stream = nullptr;
    std::vector<Level> lv;
    std::vector<void *> allocs;
    unsigned long long *d_status = nullptr;
    unsigned long long *d_norm = nullptr;  // ||A||_inf bits
    void *d_dump = nullptr;                // target of masked stores (kDumpBytes)
    // solve workspace
    int rhs_cap = 0;
    std::vector<double *> wsF, wsFadd, wsY;
    double *wsPadF = nullptr, *wsPadX = nullptr, *wsR = nullptr, *wsD = nullptr;
    unsigned long long *d_norms = nullptr;
    std::vector<void *> ws_allocs;
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
int target_rows(int M, bool f32, int level, int user)
{
    if (level == 0 && user > 0) return user;
    (void)f32;
    if (level == 0) return M <= 4 ? 16 : (M <= 8 ? 8 : 4);
    return 4;
}

constexpr int64_t kTail = 6;   // block tridiagonal systems this small: one chain

std::vector<PlanLevel> make_plan(int kind, int64_t nb, int M, const pf_opts &o)
{
    std::vector<PlanLevel> out;
    const bool f32 = o.prec == PF_FP32_IR;
    int64_t cur = nb;
    int lvl = 0;
    if (kind == PF_BABD) {
        while (cur > 2) {
            int64_t p;
            if (lvl == 0 && o.partitions > 0) p = o.partitions;
            else {
                const int L = target_rows(M, f32, lvl, o.block_rows);
                p = (cur - 1) / (L + 1);
                p = std::max<int64_t>(p, 1);
                p = std::min<int64_t>(p, (cur - 1) / 2);
            }
            out.push_back({PF_BABD, cur, p});
            cur = p + 1;
            ++lvl;
        }
        out.push_back({PF_BTRI, cur, 1});
        return out;
    }
    while (true) {
        int64_t p;
        if (lvl == 0 && o.partitions > 0) p = o.partitions;
        else if (cur <= kTail) p = 1;
        else {
            const int L = target_rows(M, f32, lvl, o.block_rows);
            p = (cur + 1) / (L + 1);
            p = std::max<int64_t>(p, 2);
            p = std::min<int64_t>(p, (cur + 1) / 2);
        }
        out.push_back({PF_BTRI, cur, p});
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

hipError_t dalloc(pf_factor_s *F, void **p, size_t bytes, std::vector<void *> &list)
{
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMallocAsync(p, bytes, F->stream);
    if (e != hipSuccess) { *p = nullptr; return e; }
    list.push_back(*p);
    return hipSuccess;
}

void free_list(pf_factor_s *F, std::vector<void *> &list)
{
    for (void *p : list) hipFreeAsync(p, F->stream);
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
    if (o.partitions < 0 || o.block_rows < 0) return -2;
    if (o.partitions > 0) {
        const int64_t pmax = (A->kind == PF_BTRI) ? (A->nb + 1) / 2 : (A->nb - 1) / 2;
        if (o.partitions > pmax && !(A->kind == PF_BABD && A->nb == 2)) return -2;
    }
    return 0;
}

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return PF_EHIP;       \
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
    hipError_t e = hipEventRecord(sl.a, s);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    return hipEventRecord(sl.b, s);
}

hipError_t launch_factor_levels(pf_factor_s *F, hipStream_t s)
{
    F->prof_fac_n = 0;
    hipError_t e = launch_fill_u64(F->d_status, 1, ~0ull, s);
    if (e != hipSuccess) return e;
    if (F->M != F->m) {
        const pf_matrix &A0 = F->A;
        e = launch_pad_blocks(A0.m, F->M, A0.nb, A0.D, F->padD, 1.0, s);
        if (e == hipSuccess) e = launch_pad_blocks(A0.m, F->M, A0.nb - 1, A0.Lo, F->padLo, 0.0, s);
        if (e == hipSuccess && F->padUp)
            e = launch_pad_blocks(A0.m, F->M, A0.nb - 1, A0.Up, F->padUp, 0.0, s);
        if (e == hipSuccess && F->padC) e = launch_pad_blocks(A0.m, F->M, 1, A0.C, F->padC, 0.0, s);
        if (e != hipSuccess) return e;
    }
    for (size_t l = 0; l < F->lv.size(); ++l) {
        const Level &L = F->lv[l];
        LevelArgs a{};
        a.nb = L.nb; a.p = L.p;
        a.D = L.D; a.Dadd = L.Dadd; a.Lo = L.Lo; a.Up = L.Up; a.C = L.C;
        a.E = L.E; a.R = L.R; a.Z = L.Z; a.X = L.X;
        a.nD = L.nD; a.nDadd = L.nDadd; a.nLo = L.nLo; a.nUp = L.nUp; a.nC = L.nC;
        a.status = F->d_status;
        a.dump = F->d_dump;
        a.level = (int)l;
        e = prof_launch(F, true, 0, (int)l, s, [&] {
            return (L.kind == PF_BTRI) ? launch_btri_factor(F->M, L.f32, a, s)
                                       : launch_babd_factor(F->M, L.f32, a, s);
        });
        if (e != hipSuccess) return e;
    }
    const pf_matrix *A = &F->A;
    if (F->opts.prec == PF_FP32_IR || (F->opts.flags & PF_FLAG_ETA)) {
        e = launch_fill_u64(F->d_norm, 1, 0ull, s);
        if (e != hipSuccess) return e;
        e = launch_norminf(A->kind, A->m, A->nb, A->D, A->Lo, A->Up, A->C, F->d_norm, s);
    }
    return e;
}

int ensure_workspace(pf_factor_s *F, int nrhs)
{
    if (nrhs <= F->rhs_cap) return 0;
    free_list(F, F->ws_allocs);
    const int cap = std::max(nrhs, 1);
    const size_t L = F->lv.size();
    F->wsF.assign(L, nullptr);
    F->wsFadd.assign(L, nullptr);
    F->wsY.assign(L, nullptr);
    for (size_t l = 1; l < L; ++l) {
        const size_t bytes = (size_t)F->lv[l].nb * F->M * cap * sizeof(double);
        void *p;
        if (dalloc(F, &p, bytes, F->ws_allocs) != hipSuccess) return PF_ENOMEM;
        F->wsF[l] = (double *)p;
        if (F->lv[l - 1].kind == PF_BTRI) {
            if (dalloc(F, &p, bytes, F->ws_allocs) != hipSuccess) return PF_ENOMEM;
            F->wsFadd[l] = (double *)p;
        }
        if (dalloc(F, &p, bytes, F->ws_allocs) != hipSuccess) return PF_ENOMEM;
        F->wsY[l] = (double *)p;
    }
    const size_t nP = (size_t)F->nb * F->M * cap * sizeof(double);
    const size_t n = (size_t)F->nb * F->m * cap * sizeof(double);
    void *p;
    if (F->M != F->m) {
        if (dalloc(F, &p, nP, F->ws_allocs) != hipSuccess) return PF_ENOMEM;
        F->wsPadF = (double *)p;
        if (dalloc(F, &p, nP, F->ws_allocs) != hipSuccess) return PF_ENOMEM;
        F->wsPadX = (double *)p;
    }
    if (dalloc(F, &p, n, F->ws_allocs) != hipSuccess) return PF_ENOMEM;
    F->wsR = (double *)p;
    if (dalloc(F, &p, n, F->ws_allocs) != hipSuccess) return PF_ENOMEM;
    F->wsD = (double *)p;
    if (dalloc(F, &p, 3 * (size_t)cap * sizeof(unsigned long long), F->ws_allocs) != hipSuccess)
        return PF_ENOMEM;
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
    std::vector<SolveArgs> args(L);
    for (size_t l = 0; l < L; ++l) {
        const Level &lv = F->lv[l];
        SolveArgs &a = args[l];
        a = SolveArgs{};
        a.nb = lv.nb;
        a.dump = (double *)F->d_dump;
        a.p = lv.p;
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
    F->prof_sol_n = 0;
    for (size_t l = 0; l < L; ++l) {
        const Level &lv = F->lv[l];
        HIPCHK(prof_launch(F, false, 1, (int)l, s, [&] {
            return lv.kind == PF_BTRI ? launch_btri_fwd(M, lv.f32, args[l], s)
                                      : launch_babd_fwd(M, lv.f32, args[l], s);
        }));
    }
    for (size_t l = L; l-- > 0;) {
        const Level &lv = F->lv[l];
        HIPCHK(prof_launch(F, false, 2, (int)l, s, [&] {
            return lv.kind == PF_BTRI ? launch_btri_bwd(M, lv.f32, args[l], s)
                                      : launch_babd_bwd(M, lv.f32, args[l], s);
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
int compute_eta(pf_factor_s *F, int nrhs, const double *f, int64_t ldf, const double *x,
                int64_t ldx, double *r, int64_t ldr, hipStream_t s, double *eta_out)
{
    const pf_matrix &A = F->A;
    HIPCHK(launch_fill_u64(F->d_norms, 3 * nrhs, 0ull, s));
    HIPCHK(launch_residual(A.kind, A.m, A.nb, A.D, A.Lo, A.Up, A.C, nrhs, f, ldf, x, ldx, r, ldr,
                           F->d_norms, s));
    std::vector<unsigned long long> h(3 * nrhs + 1);
    HIPCHK(hipMemcpyAsync(h.data(), F->d_norms, 3 * nrhs * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h.data() + 3 * nrhs, F->d_norm, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
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
    *eta_out = worst;
    return 0;
}

void read_status(pf_factor_s *F, pf_info *info)
{
    unsigned long long st = ~0ull;
    hipMemcpy(&st, F->d_status, sizeof st, hipMemcpyDeviceToHost);
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
    default: return "unknown error";
    }
}

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
    b += 2 * (size_t)A->nb * A->m * 8 + 24;
    return b;
}

int pf_factor(const pf_matrix *A, const pf_opts *opts, void *stream, pf_factor_t *out)
{
    if (!out) return -4;
    *out = nullptr;
    int rc = check_matrix(A);
    if (rc) return rc;
    const pf_opts o = resolve_opts(opts);
    if ((rc = check_opts(A, o))) return rc;

    pf_factor_s *F = new pf_factor_s();
    F->A = *A;
    F->opts = o;
    F->m = A->m;
    F->M = padded_block(A->m);
    F->nb = A->nb;
    F->stream = (hipStream_t)stream;
    const int M = F->M;
    const size_t bd = (size_t)M * M * sizeof(double);
    hipStream_t s = F->stream;
    auto fail = [&](int code) {
        free_list(F, F->allocs);
        hipStreamSynchronize(s);
        delete F;
        return code;
    };
    void *p;
    if (dalloc(F, &p, 2 * sizeof(unsigned long long), F->allocs) != hipSuccess)
        return fail(PF_ENOMEM);
    F->d_status = (unsigned long long *)p;
    F->d_norm = F->d_status + 1;
    if (dalloc(F, &F->d_dump, kDumpBytes, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
    if (launch_fill_u64(F->d_status, 1, ~0ull, s) != hipSuccess) return fail(PF_EHIP);
    if (launch_fill_u64(F->d_norm, 1, 0ull, s) != hipSuccess) return fail(PF_EHIP);

    // level-0 matrix (padded to an instantiated block size if needed; the
    // padding itself runs in launch_factor_levels so refactor redoes it)
    const double *D0 = A->D, *Lo0 = A->Lo, *Up0 = A->Up, *C0 = A->C;
    if (M != A->m) {
        if (dalloc(F, &p, A->nb * bd, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
        F->padD = (double *)p;
        if (dalloc(F, &p, (A->nb - 1) * bd, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
        F->padLo = (double *)p;
        D0 = F->padD;
        Lo0 = F->padLo;
        if (A->kind == PF_BTRI) {
            if (dalloc(F, &p, (A->nb - 1) * bd, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
            F->padUp = (double *)p;
            Up0 = F->padUp;
        } else {
            if (dalloc(F, &p, bd, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
            F->padC = (double *)p;
            C0 = F->padC;
        }
    }

    const auto plan = make_plan(A->kind, A->nb, M, o);
    F->lv.resize(plan.size());
    for (size_t l = 0; l < plan.size(); ++l) {
        Level &L = F->lv[l];
        L.kind = plan[l].kind;
        L.nb = plan[l].nb;
        L.p = plan[l].p;
        L.f32 = (l == 0 && o.prec == PF_FP32_IR);
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
        if (dalloc(F, &L.E, fb, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
        if (dalloc(F, &L.Z, fb, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
        if (L.kind == PF_BTRI) {
            if (dalloc(F, &L.R, fb, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
            if (dalloc(F, &L.X, fb, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
            if (L.p > 1) {
                const size_t rb = (size_t)(L.p - 1) * bd;
                if (dalloc(F, &p, rb, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
                L.nD = (double *)p;
                if (dalloc(F, &p, rb, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
                L.nDadd = (double *)p;
                if (dalloc(F, &p, rb, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
                L.nLo = (double *)p;
                if (dalloc(F, &p, rb, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
                L.nUp = (double *)p;
            }
        } else {
            if (dalloc(F, &p, (size_t)(L.p + 1) * bd, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
            L.nD = (double *)p;
            if (dalloc(F, &p, (size_t)L.p * bd, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
            L.nLo = (double *)p;
            if (dalloc(F, &p, bd, F->allocs) != hipSuccess) return fail(PF_ENOMEM);
            L.nC = (double *)p;
        }
    }
    if (launch_factor_levels(F, s) != hipSuccess) return fail(PF_EHIP);
    *out = F;
    return 0;
}

int pf_refactor(pf_factor_t F, void *stream)
{
    if (!F) return -1;
    hipStream_t s = stream ? (hipStream_t)stream : F->stream;
    return launch_factor_levels(F, s) == hipSuccess ? 0 : PF_EHIP;
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

int pf_solve(pf_factor_t F, int32_t nrhs, const double *f, int64_t ldf, double *x, int64_t ldx,
             void *stream, pf_info *info)
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
    if (F->opts.prec == PF_FP64) {
        if ((rc = run_solve(F, nrhs, f, ldf, x, ldx, s))) return rc;
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
    if ((rc = run_solve(F, nrhs, f, ldf, x, ldx, s))) return rc;
    double eta = INFINITY, prev = INFINITY;
    int iters = 0, slow = 0, status = PF_OK;
    for (;;) {
        if ((rc = compute_eta(F, nrhs, f, ldf, x, ldx, F->wsR, n, s, &eta))) return rc;
        if (eta <= F->opts.tol) break;
        if (iters >= F->opts.max_refine) { status = PF_ENOCONV; break; }
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

void pf_destroy(pf_factor_t F)
{
    if (!F) return;
    free_list(F, F->ws_allocs);
    free_list(F, F->allocs);
    hipStreamSynchronize(F->stream);
    for (auto *list : {&F->prof_fac, &F->prof_sol})
        for (auto &sl : *list) {
            if (sl.a) hipEventDestroy(sl.a);
            if (sl.b) hipEventDestroy(sl.b);
        }
    delete F;
}

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

int pf_solve_batch(int32_t nsys, const pf_matrix *A, const pf_opts *opts, const int32_t *nrhs,
                   const double *const *f, const int64_t *ldf, double *const *x,
                   const int64_t *ldx, void *stream, pf_factor_t *factors, pf_info *info)
{
    if (nsys < 0) return -1;
    if (nsys > 0 && !A) return -2;
    if (nsys > 0 && (!nrhs || !f || !ldf || !x || !ldx)) return -4;
    int worst = 0;
    for (int i = 0; i < nsys; ++i) {
        pf_factor_t Fi = nullptr;
        int rc = pf_factor(&A[i], opts, stream, &Fi);
        if (rc) {
            if (info) { std::memset(&info[i], 0, sizeof(pf_info)); info[i].status = rc; }
            worst = worst ? worst : rc;
            if (factors) factors[i] = nullptr;
            continue;
        }
        pf_info inf{};
        rc = pf_solve(Fi, nrhs[i], f[i], ldf[i], x[i], ldx[i], stream, info ? &inf : nullptr);
        if (info) info[i] = inf;
        if (rc && !worst) worst = rc;
        if (factors) factors[i] = Fi;
        else pf_destroy(Fi);
    }
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PF_EHIP;
    return worst;
}

}  // extern "C"
