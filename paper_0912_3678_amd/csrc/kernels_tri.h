// Scalar tridiagonal levels (m = 1, FP64) with coalesced HBM access: host-side
// launchers of kernels_tri.hip.
//
// Each workgroup (one wave) owns 64 consecutive partitions of a level and
// stages their rows, through their right separators, in LDS with contiguous
// loads; each lane then runs its partition's chain (the recurrences of the
// block factorization, Sec. 2, with 1 x 1 blocks) out of LDS, and the
// workgroup writes the per-row factors back contiguously.  The stored factors
// of the partitions' rows and the reduced system are those of the segment
// mapping with one entry per lane, bit for bit, so the forward sweep and the
// batched kernels read them unchanged (the separators' rows of the factor
// arrays, which no kernel reads, hold other values).
#pragma once
#include <hip/hip_runtime.h>

#include "pf_internal.h"

namespace pf {

// longest partition (blocks) a workgroup's LDS holds
constexpr int kTriMaxChain = 17;

// whether a level of nb rows in p partitions fits the kernels' LDS
bool tri_fits(int64_t nb, int64_t p);

// factor of a block tridiagonal level with m = 1 (FP64); with sv != NULL
// (sv->nrhs == 1) the forward sweep runs in the same pass.  a.Dadd (and
// sv->Fadd) select the two-addend form of the reduced levels.
hipError_t launch_tri_factor(const LevelArgs &a, const SolveArgs *sv, hipStream_t s);

// forward sweep of a block tridiagonal level with m = 1 (stored factors), one
// right-hand side, FP64 factors; sv.Fadd selects the two-addend form
hipError_t launch_tri_fwd(const SolveArgs &a, hipStream_t s);

// back substitution of a block tridiagonal level with m = 1, one right-hand
// side, FP64 factors
hipError_t launch_tri_bwd(const SolveArgs &a, hipStream_t s);

// A whole scalar tridiagonal system (nb rows, p partitions) in one launch of
// one workgroup (kernels_tri_cr.hip): local cyclic reduction of the
// partitions, parallel cyclic reduction of the reduced system across a
// wave, back substitution; one right-hand side, FP64, no pivoting.
constexpr int kTriCrMaxRows = 4096;   // rows in LDS (4 words each)
constexpr int kTriCrMaxParts = 64;    // reduced system: one wave's lanes
bool tri_cr_fits(int64_t nb, int64_t p);
hipError_t launch_tri_cr_whole(int64_t nb, int64_t p, const double *D, const double *Lo,
                               const double *Up, const double *f, double *x,
                               unsigned long long *status, hipStream_t s);

}  // namespace pf
