// sign(A) of general square matrices of small order: the kernels' interface
// (csrc/signm.hip), used by the batched entry point in csrc/api.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sgt {

struct cd;  // complex double (re, im)

// Largest order the one-wave Schur kernels take (A's Hessenberg and Schur
// forms in LDS).
constexpr int kSignmMaxOrder = 64;

// One matrix of a batch: device pointers, column-major, leading dimensions.
// Real matrices are doubles, complex ones interleaved (re, im) pairs.
struct SignmMat {
    const double *A;
    double *S;
    int64_t lda, lds;
    int32_t n;
    int32_t index;  // position in the caller's batch (for the status word)
    cd *Q;          // n x n complex workspace for Q (row-major)
};

// Per-matrix outcome written by the kernels.
enum { SIGNM_OK = 0, SIGNM_EDOMAIN = 1, SIGNM_ENOCONV = 4 };

// Launch the Schur kernels over mats[0, count): matrices of order at most 32
// first (smaller LDS, more workgroups per compute unit), then the rest; the
// table must be sorted that way, with n32 of them of order at most 32.
// status[index] receives each matrix's outcome.
// max_sweeps > 0 replaces the QR iteration's limit of 30 max(10, n) sweeps (a
// testing hook: a tiny limit makes the not-converged report reachable).
hipError_t launch_signm(const SignmMat *mats, int count, int n32, bool cplx, int32_t *status,
                        int max_sweeps, hipStream_t st);

}  // namespace sgt
