// Scalar tridiagonal systems small enough for one workgroup's LDS, solved by
// the partition method in one launch: the p partitions are eliminated by
// local cyclic reduction (the cyclic-reduction variant of the local
// factorization in Sec. 2: the rounds halve a partition's rows while its two
// boundary rows are kept, and no fill-in vectors are formed), the reduced
// tridiagonal system on the p - 1 separators (eq. (redmatr)) is solved by
// parallel cyclic reduction across one wave's lanes with cross-lane
// shuffles, and the partitions are back-substituted through their rounds in
// reverse.  No pivoting (as cyclic reduction itself): a zero pivot is
// reported like the other factor kernels' (status word, level 0 for a
// partition's row, level 1 for a separator).
//
// Layout: the rows' a = A(g, g-1), b = A(g, g), c = A(g, g+1) and f live in
// LDS for the whole solve (4 x 8 bytes per row), partition by partition,
// each partition's run framed by copies of its two boundary rows (the left
// separator's row as seen from this partition starts with b = f = 0 and
// collects this partition's contribution; the right separator's row starts
// from D and f of the separator), so partitions sharing a separator never
// write the same word.
#include "kernels_tri.h"
#include "kernels_common.h"

namespace pf {
namespace {

constexpr int kCrThreads = 1024;

__global__ __launch_bounds__(kCrThreads) void k_tri_cr_whole(int nb, int p, const double *D,
                                                             const double *Lo, const double *Up,
                                                             const double *f, double *x,
                                                             unsigned long long *status)
{
    // partition i's local positions 0 .. n_i + 1 are the words base_i ..
    // base_i + n_i + 1 of each array (base_i = start_i + i, so the frames
    // lie back to back): its boundary rows are copies of its own, so every
    // access is a plain index
    constexpr int W = kTriCrMaxRows + kTriCrMaxParts + 1;
    __shared__ double A[W], B[W], C[W], F[W];
    __shared__ double xs[kTriCrMaxParts + 1];   // separator solutions (xs[j]: separator j, 1-based)
    __shared__ unsigned long long sbad;
    const int tid = threadIdx.x;
    if (tid == 0) sbad = ~0ull;
    // interior rows, by partition: row g of partition i sits at g + i + 1.
    // Balanced rule in 32 bits: the first rem partitions take q + 1 rows
    // and their separator, the others q rows and theirs.
    const int nint = nb - (p - 1), q = nint / p, rem = nint - q * p;
    const int big = rem * (q + 2);
    auto part_of = [&](int g) { return g < big ? g / (q + 2) : rem + (g - big) / (q + 1); };
    auto start_of = [&](int i) { return i * (q + 1) + (i < rem ? i : rem); };
    auto len_of = [&](int i) { return q + (i < rem ? 1 : 0); };
    constexpr int RPT = kTriCrMaxRows / kCrThreads;   // rows per thread
    {
        // every load of the thread first (independent), then the LDS stores
        double va[RPT], vb[RPT], vc[RPT], vf[RPT];
#pragma unroll
        for (int it = 0; it < RPT; ++it) {
            const int g = tid + it * kCrThreads;
            const bool ok = g < nb;
            va[it] = (ok && g > 0) ? Lo[g - 1] : 0.0;
            vb[it] = ok ? D[g] : 0.0;
            vc[it] = (ok && g + 1 < nb) ? Up[g] : 0.0;
            vf[it] = ok ? f[g] : 0.0;
        }
#pragma unroll
        for (int it = 0; it < RPT; ++it) {
            const int g = tid + it * kCrThreads;
            if (g >= nb) continue;
            const int i = part_of(g), st = start_of(i), ln = len_of(i);
            const int base = st + i;
            if (g < st + ln) {          // an interior row of partition i
                const int k = base + (g - st) + 1;
                A[k] = va[it]; B[k] = vb[it]; C[k] = vc[it]; F[k] = vf[it];
            } else {                    // separator g: right boundary of i, left of i + 1
                const int kr = base + ln + 1, kl = kr + 1;
                A[kr] = va[it]; B[kr] = vb[it]; C[kr] = 0.0; F[kr] = vf[it];
                A[kl] = 0.0; B[kl] = 0.0; C[kl] = vc[it]; F[kl] = 0.0;
            }
        }
    }
    const int tpp = kCrThreads / p;
    const int part = tid / tpp, lt = tid % tpp;
    // partitions that each lie within one wave (16, 32 or 64 of them, and
    // up to 64 lanes each) need only their own wave's ordering between the
    // rounds; the workgroup meets where the reduced system is formed
    const bool wave_local = 64 % tpp == 0;   // uniform
    auto round_sync = [&]() {
        if (wave_local) wave_sync();
        else __syncthreads();
    };
    const bool mine = part < p;
    const int pm = mine ? part : 0;
    const bool hasL = mine && part > 0, hasR = mine && part < p - 1;
    const int s0 = start_of(pm), n = mine ? len_of(pm) : 0, base = s0 + pm;
    if (mine && lt == 0) {
        // no left separator (first partition) / right one (last): null rows
        if (!hasL) { A[base] = 0.0; B[base] = 0.0; C[base] = 0.0; F[base] = 0.0; }
        if (!hasR) {
            const int kr = base + n + 1;
            A[kr] = 0.0; B[kr] = 1.0; C[kr] = 0.0; F[kr] = 0.0;
        }
    }
    __syncthreads();

    // rounds: at round r (h = 2^(r-1)) the active positions are the
    // multiples of h up to n and n + 1; the odd multiples are eliminated,
    // each survivor (a multiple of 2h, or n + 1) folds in its eliminated
    // neighbours: with l its left and q its right neighbour,
    //   b -= (a / b_l) c_l + (c / b_q) a_q,  f -= (a / b_l) f_l + (c / b_q) f_q,
    //   a <- -(a / b_l) a_l,  c <- -(c / b_q) c_q.
    // A survivor reads only its own row and its eliminated neighbours, which
    // no thread writes in the round, and writes only its own row: the
    // survivors of a round are updated in place, in any order.
    int rounds = 0;
    while ((1 << rounds) <= n) ++rounds;                       // this partition's
    int rmax = 0;
    while ((1 << rmax) <= (nb + p - 1) / p + 1) ++rmax;        // every partition's bound
    unsigned long long bad = ~0ull;
    for (int r = 1; r <= rmax; ++r) {
        const int h = 1 << (r - 1);
        if (mine && r <= rounds) {
            const int cnt = n / (2 * h) + 2;   // survivors: 0, 2h, 4h, ... <= n, and n + 1
            for (int i = lt; i < cnt; i += tpp) {
                const int jj = (i == cnt - 1) ? n + 1 : 2 * h * i;
                // eliminated neighbours: jj - h and jj + h for a multiple of
                // 2h; for n + 1 the largest multiple of h <= n when it is odd
                int l = -1, q = -1;
                if (jj == n + 1) {
                    const int L = (n / h) * h;
                    if (L >= 1 && ((L / h) & 1)) l = L;
                } else {
                    if (jj >= h) l = jj - h;
                    if (jj + h <= n) q = jj + h;
                }
                const int kj = base + jj;
                double a = A[kj], b = B[kj], c = C[kj], ff = F[kj];
                if (l >= 1) {
                    const int kl = base + l;
                    const double bl = B[kl];
                    bad = (bl == 0.0) ? min(bad, status_code(0, s0 + l - 1)) : bad;
                    const double k1 = a * recip(bl);
                    b -= k1 * C[kl];
                    ff -= k1 * F[kl];
                    a = -k1 * A[kl];
                }
                if (q >= 1) {
                    const int kq = base + q;
                    const double bq = B[kq];
                    bad = (bq == 0.0) ? min(bad, status_code(0, s0 + q - 1)) : bad;
                    const double k2 = c * recip(bq);
                    b -= k2 * A[kq];
                    ff -= k2 * F[kq];
                    c = -k2 * C[kq];
                }
                A[kj] = a; B[kj] = b; C[kj] = c; F[kj] = ff;
            }
        }
        round_sync();
    }
    __syncthreads();

    // the reduced system on the separators: row j (separator j = right
    // boundary of partition j - 1 and left boundary of partition j), by
    // parallel cyclic reduction across the lanes of wave 0 (lane i: row i+1)
    if (tid < 64) {
        const int i = tid + 1;
        const bool real = i <= p - 1;
        int kr = 0, kl = 0;
        if (real) {
            kr = start_of(i - 1) + (i - 1) + len_of(i - 1) + 1;   // right boundary of partition i - 1
            kl = kr + 1;                                          // left boundary of partition i
        }
        double a = real && i > 1 ? A[kr] : 0.0;            // beta
        double b = real ? B[kr] + B[kl] : 1.0;             // D + alpha_2 + alpha_1
        double c = real && i < p - 1 ? C[kl] : 0.0;        // gamma
        double ff = real ? F[kr] + F[kl] : 0.0;
        for (int st = 1; st < 64; st <<= 1) {
            const int lo = tid - st, hi = tid + st;
            const double al = __shfl(a, lo < 0 ? tid : lo), bl = __shfl(b, lo < 0 ? tid : lo),
                         cl = __shfl(c, lo < 0 ? tid : lo), fl = __shfl(ff, lo < 0 ? tid : lo);
            const double ah = __shfl(a, hi > 63 ? tid : hi), bh = __shfl(b, hi > 63 ? tid : hi),
                         ch = __shfl(c, hi > 63 ? tid : hi), fh = __shfl(ff, hi > 63 ? tid : hi);
            const bool hl = lo >= 0, hh = hi <= 63;
            bad = (real && ((hl && bl == 0.0) || (hh && bh == 0.0)))
                      ? min(bad, status_code(1, i - 1)) : bad;
            const double k1 = hl ? a * recip(bl) : 0.0, k2 = hh ? c * recip(bh) : 0.0;
            const double na2 = hl ? -k1 * al : 0.0, nc2 = hh ? -k2 * ch : 0.0;
            b = b - (hl ? k1 * cl : 0.0) - (hh ? k2 * ah : 0.0);
            ff = ff - (hl ? k1 * fl : 0.0) - (hh ? k2 * fh : 0.0);
            a = na2;
            c = nc2;
        }
        bad = (real && b == 0.0) ? min(bad, status_code(1, i - 1)) : bad;
        if (real) {
            const double v = ff / b;
            xs[i] = v;
            F[kr] = v;   // the separator's solution, where the store below finds it
        }
    }
    __syncthreads();

    // back substitution through the rounds in reverse: an eliminated row l
    // of round r has x_l = (f_l - a_l x_{l-h} - c_l x_{l+h or n+1}) / b_l,
    // its neighbours solved in a later round; x overwrites f (the boundary
    // positions first take their separator's solution)
    if (mine && lt == 0) {
        F[base] = hasL ? xs[part] : 0.0;
        F[base + n + 1] = hasR ? xs[part + 1] : 0.0;
    }
    __syncthreads();
    for (int r = rmax; r >= 1; --r) {
        const int h = 1 << (r - 1);
        if (mine && r <= rounds) {
            const int cnt = (n + h) / (2 * h);   // odd multiples of h <= n
            for (int i = lt; i < cnt; i += tpp) {
                const int l = (2 * i + 1) * h;
                const int q = l + h <= n ? l + h : n + 1;
                const int kl = base + l;
                F[kl] = (F[kl] - A[kl] * F[base + l - h] - C[kl] * F[base + q]) * recip(B[kl]);
            }
        }
        round_sync();
    }
    if (bad != ~0ull) atomicMin(&sbad, bad);
    __syncthreads();
    // the status word: this launch is the whole solve, so it sets the word
    // (the first zero pivot, or none) instead of folding into it
    if (tid == 0) *status = sbad;
#pragma unroll
    for (int it = 0; it < RPT; ++it) {
        const int g = tid + it * kCrThreads;
        if (g >= nb) continue;
        const int i = part_of(g), st = start_of(i), ln = len_of(i);
        const int bi = st + i;
        // interior row: its position; separator: the right boundary of i
        x[g] = F[g < st + ln ? bi + (g - st) + 1 : bi + ln + 1];
    }
}

}  // namespace

bool tri_cr_fits(int64_t nb, int64_t p)
{
    return nb >= 2 && nb <= kTriCrMaxRows && p >= 1 && p <= kTriCrMaxParts && p <= (nb + 1) / 2;
}

hipError_t launch_tri_cr_whole(int64_t nb, int64_t p, const double *D, const double *Lo,
                               const double *Up, const double *f, double *x,
                               unsigned long long *status, hipStream_t s)
{
    if (!tri_cr_fits(nb, p)) return hipErrorInvalidValue;
    launch_k(k_tri_cr_whole, dim3(1), dim3(kCrThreads), s, (int)nb, (int)p, D, Lo, Up, f, x,
             status);
    return hipGetLastError();
}

}  // namespace pf
