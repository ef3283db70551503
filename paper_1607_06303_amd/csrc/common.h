// Internal declarations shared by the HIP sources of libsigntri.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/signtri.h"

namespace sgt {

// ---------------------------------------------------------------------------
// Scalars.  Complex numbers are interleaved (re, im) doubles, as in the ABI.
// ---------------------------------------------------------------------------
struct cd {
    double re, im;
};

__host__ __device__ inline cd operator+(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cd operator-(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cd operator-(cd a) { return {-a.re, -a.im}; }
__host__ __device__ inline cd operator*(cd a, cd b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cd operator*(cd a, double x) { return {a.re * x, a.im * x}; }
__host__ __device__ inline cd operator/(cd a, cd b)
{
    double den = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
__host__ __device__ inline cd operator/(cd a, double x) { return {a.re / x, a.im / x}; }

template <typename S> struct scalar_traits;
template <> struct scalar_traits<double> {
    __host__ __device__ static double zero() { return 0.0; }
    __host__ __device__ static double from_real(double x) { return x; }
    __host__ __device__ static double real(double x) { return x; }
    __device__ static double shfl_xor(double v, int m) { return __shfl_xor(v, m, 64); }
};
template <> struct scalar_traits<float> {
    __host__ __device__ static float zero() { return 0.0f; }
    __host__ __device__ static float from_real(double x) { return (float)x; }
    __host__ __device__ static double real(float x) { return x; }
    __device__ static float shfl_xor(float v, int m) { return __shfl_xor(v, m, 64); }
};
template <> struct scalar_traits<cd> {
    __host__ __device__ static cd zero() { return {0.0, 0.0}; }
    __host__ __device__ static cd from_real(double x) { return {x, 0.0}; }
    __host__ __device__ static double real(cd x) { return x.re; }
    __device__ static cd shfl_xor(cd v, int m)
    {
        return {__shfl_xor(v.re, m, 64), __shfl_xor(v.im, m, 64)};
    }
};

// ---------------------------------------------------------------------------
// MFMA wrappers (gfx950).  For both 16x16x4 shapes, lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Element r of the accumulator
// holds D[row][l % 16] with row = l / 16 + 4 r for the f64 instruction and
// row = 4 (l / 16) + r for the f32 one (measured on the device).
// ---------------------------------------------------------------------------
typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

__device__ inline int mfma64_row(int lane, int r) { return (lane >> 4) + 4 * r; }
__device__ inline int mfma32_row(int lane, int r) { return 4 * (lane >> 4) + r; }

__device__ inline dx4 mfma_f64(double a, double b, dx4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline fx4 mfma_f32(float a, float b, fx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Device-side plan data: per-index sign (+1/-1) and scan results.
// ---------------------------------------------------------------------------
struct ScanResult {
    int64_t bad_index;  // smallest 0-based index with an undefined sign, or n
    int64_t n_pos;
};

// Host planner (Section 3), shared by signtri() and signtri_plan_host().
struct HostPlan {
    int64_t n_pos = 0, n_neg = 0;
    int64_t swaps_pos_first = 0, swaps_neg_first = 0;
    double w_ph = 0, w_ps = 0;
    int model_pick = SIGNTRI_PATH_PH;
    int auto_path = SIGNTRI_PATH_PH;
    int ps_sign = 0;  // +1: positives first, -1: negatives first, 0: not grouped
    int64_t split = 0;  // size of the leading sign group when grouped
};
HostPlan plan_from_signs(const int8_t *s, int64_t n, bool is_complex);

// ---------------------------------------------------------------------------
// Opt-in kernel timers: when enabled, every launch is bracketed by a pair of
// HIP events on its stream and credited to a kernel family together with the
// algorithmic flops (Section 3 counting) of the work it does.
// ---------------------------------------------------------------------------
enum ProfKind {
    PK_SCAN = 0,
    PK_DIAG = 1,
    PK_GEMM = 2,
    PK_SOLVE = 3,
    PK_AUX = 4,
    PK_RESID = 5,
    PK_CORR_GEMM = 6,
    PK_CORR_SOLVE = 7,
    PK_SYL_GEMM = 8,
    PK_SYL_SOLVE = 9,
    PK_BATCHED = 10,
    PK_CONVERT = 11,
    PK_COUNT = 16
};
bool prof_on();
void prof_begin(hipStream_t st);
void prof_end(hipStream_t st, int kind, double flops);

// ---------------------------------------------------------------------------
// Launchers (each in its own translation unit).
// ---------------------------------------------------------------------------
hipError_t launch_scan(const void *T, int64_t ldt, int64_t n, bool cplx, int8_t *sgn,
                       ScanResult *res, hipStream_t st);
hipError_t launch_zero_lower(void *U, int64_t ldu, int64_t n, bool cplx, hipStream_t st);
hipError_t launch_fill_pm_identity(void *U, int64_t ldu, int64_t n, bool cplx, double s,
                                   hipStream_t st);

// Parlett-Higham block sweep, FP64 (real: tile 64, complex: tile 32).
struct PhArgs {
    const void *T;
    int64_t ldt;
    void *U;
    int64_t ldu;
    int64_t n;
    const int8_t *sgn;
    const int8_t *hsgn;  // the same signs in host memory (flop accounting)
    void *zbuf;          // block accumulators: zslots * tile * tile scalars
    int64_t zslots;
    int max_splits;
};
int ph_tile_size(bool cplx);
int64_t ph_zslots(int64_t n, bool cplx);
hipError_t run_ph_fp64(const PhArgs &a, bool cplx, hipStream_t st);

}  // namespace sgt
