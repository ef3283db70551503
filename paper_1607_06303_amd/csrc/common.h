// Internal declarations shared by the HIP sources of libsigntri.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>
#include <vector>

#include "../../include/signtri.h"

namespace sgt {

constexpr int kLookahead = 3;  // bulk products run kLookahead-1 superdiagonals ahead

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
    // a conj(b) / |b|^2 with b scaled by max(|Re b|, |Im b|), so that |b|^2 neither
    // overflows nor underflows (and a power-of-two scaling of a and b passes through
    // exactly)
    const double s = fmax(fabs(b.re), fabs(b.im));
    const double xr = b.re / s, xi = b.im / s;
    const double den = s * (xr * xr + xi * xi);
    return {(a.re * xr + a.im * xi) / den, (a.im * xr - a.re * xi) / den};
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

// Sum over aligned groups of 8 consecutive lanes with DPP moves (no LDS):
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], then row_half_mirror.
// Every lane reads a valid source lane in these patterns (all rows and banks
// enabled), so the move needs no prior value in its destination.
template <int CTRL> __device__ inline float dppf(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL> __device__ inline double dppd(double v)
{
    long long b = __double_as_longlong(v);
    int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double group8_sum(double v)
{
    v += dppd<0xB1>(v);
    v += dppd<0x4E>(v);
    v += dppd<0x141>(v);
    return v;
}
__device__ inline float group8_sum(float v)
{
    v += dppf<0xB1>(v);
    v += dppf<0x4E>(v);
    v += dppf<0x141>(v);
    return v;
}
// Sum over aligned groups of L consecutive lanes (L = 4, 8 or 16); every lane
// of a group receives the group's sum.  16: the 8-lane sums are combined with
// row_mirror (lane i and lane 15 - i lie in different halves).
template <int L, typename V> __device__ inline V group_sum(V v)
{
    static_assert(L == 4 || L == 8 || L == 16, "group size");
    if constexpr (sizeof(V) == 8) {
        v += dppd<0xB1>(v);
        v += dppd<0x4E>(v);
        if constexpr (L >= 8) v += dppd<0x141>(v);
        if constexpr (L >= 16) v += dppd<0x140>(v);
    } else {
        v += dppf<0xB1>(v);
        v += dppf<0x4E>(v);
        if constexpr (L >= 8) v += dppf<0x141>(v);
        if constexpr (L >= 16) v += dppf<0x140>(v);
    }
    return v;
}

// A value every lane of the wave holds, as a scalar (SGPR) value.  Every value
// that decides whether or how often a barrier is reached must be provably
// uniform: the compiler structures a loop whose trip count it sees as
// divergent per lane, and the barriers inside it then no longer pair up
// between waves.
__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline dx4 mfma_f64(double a, double b, dx4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline fx4 mfma_f32(float a, float b, fx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Accesses through a pointer that addresses device memory.  A pointer read
// from a struct is generic to the compiler, which then emits flat loads; a
// flat load counts against the LDS counter as well, so each wait for an LDS
// read also waits for every flat load in flight and a prefetch into registers
// stops overlapping the compute.  These casts make the loads global ones.
template <typename V> using gmem = __attribute__((address_space(1))) V;
template <typename V> __device__ inline V gload(const V *p)
{
    if constexpr (std::is_arithmetic<V>::value) {
        return *(const gmem<V> *)p;
    } else {  // a struct or vector type: word by word
        static_assert(sizeof(V) % 4 == 0 && alignof(V) >= 4, "gload of a struct needs whole words");
        V v;
        const gmem<int> *s = (const gmem<int> *)p;
        int *d = (int *)&v;
#pragma unroll
        for (unsigned i = 0; i < sizeof(V) / 4; ++i) d[i] = s[i];
        return v;
    }
}
template <typename V> __device__ inline void gstore(V *p, V v) { *(gmem<V> *)p = v; }
// Device-coherent (agent scope) forms, for data another workgroup of the
// running launch writes or reads.
template <typename V> __device__ inline V gload_coherent(const V *p)
{
    return __hip_atomic_load((const gmem<V> *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V> __device__ inline void gstore_coherent(V *p, V v)
{
    __hip_atomic_store((gmem<V> *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Device-side plan data: per-index sign (+1/-1) and scan results.
// ---------------------------------------------------------------------------
struct ScanResult {
    int64_t bad_index;  // smallest 0-based index with an undefined sign, or n
    int64_t n_pos;
    uint64_t absmin, absmax;  // bits of min and max |Re t_ii| (nonnegative doubles order as
                              // their bit patterns), over the entries with a defined sign
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
    int64_t n_min = 0;  // entries in the minority sign class (ties: the negatives)
    int min_sign = 0;   // sign of the minority class
    bool proj_pick = false;  // AUTO runs the projector form instead of auto_path
};
HostPlan plan_from_signs(const int8_t *s, int64_t n, bool is_complex);

// ---------------------------------------------------------------------------
// Opt-in kernel timers: when enabled, every launch is bracketed by a pair of
// HIP events on its stream and credited to a kernel family together with the
// algorithmic flops (Section 3 counting) of the work it does.
// ---------------------------------------------------------------------------
enum ProfKind {
    PK_SCAN = SIGNTRI_K_SCAN,
    PK_DIAG = SIGNTRI_K_DIAG,
    PK_GEMM = SIGNTRI_K_GEMM,
    PK_SOLVE = SIGNTRI_K_SOLVE,
    PK_AUX = SIGNTRI_K_AUX,
    PK_RESID = SIGNTRI_K_RESID,
    PK_CORR = SIGNTRI_K_CORR,
    PK_SYL = SIGNTRI_K_SYL,
    PK_FLOW = SIGNTRI_K_FLOW,
    PK_BATCHED = SIGNTRI_K_BATCHED,
    PK_CONVERT = SIGNTRI_K_CONVERT,
    PK_PROJ = SIGNTRI_K_PROJ,
    PK_PROJ_OUT = SIGNTRI_K_PROJ_OUT,
    PK_COUNT = 16
};
bool prof_on();
void prof_begin(hipStream_t st);
// launches: kernel launches between the two events (one timed record)
void prof_end(hipStream_t st, int kind, double flops, int launches = 1);

// ---------------------------------------------------------------------------
// Launchers (each in its own translation unit).
// ---------------------------------------------------------------------------
hipError_t launch_scan(const void *T, int64_t ldt, int64_t n, bool cplx, int8_t *sgn, double *dg,
                       ScanResult *res, hipStream_t st);
hipError_t launch_zero_lower(void *U, int64_t ldu, int64_t n, bool cplx, hipStream_t st);
hipError_t launch_fill_pm_identity(void *U, int64_t ldu, int64_t n, bool cplx, double s,
                                   hipStream_t st);
hipError_t launch_transpose(const void *src, int64_t lds, void *dst, int64_t ldd, int64_t n,
                            bool cplx, hipStream_t st);

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
    void *zbufs[2];      // further bulk buffers (real path)
    void *ebuf;          // edge partials (real path)
    int64_t zslots;
    int max_splits;
    int tile;            // block size: 64 or 32 (real), 32 (complex)
};

// Algorithmic flops (Section 3 counting) per launch family, from host signs: a
// pair (i, j), i < j, costs 2 (equal signs) or 4 (opposite) real flops per k
// strictly between them (x4 for complex).  Its k are attributed to the block
// products when they lie in blocks strictly between I and J (bulk: I+2 .. J-2,
// edge: I+1 and J-1) and to the solve kernels when they lie inside I or J.
struct FlopCounter {
    const int8_t *s;
    int64_t n;
    int tb;
    double c;  // 1 real, 4 complex

    void counts(int64_t i0, int len, int64_t &pos, int64_t &neg) const
    {
        pos = neg = 0;
        for (int t = 0; t < len; ++t) (s[i0 + t] > 0 ? pos : neg)++;
    }
    // flops of the middle K blocks of superdiagonal D, per K block
    double per_k_block(int D) const
    {
        const int64_t nb = (n + tb - 1) / tb;
        double f = 0.0;
        for (int64_t I = 0; I + D < nb; ++I) {
            int64_t J = I + D;
            int bj = (int)((n - J * tb) < tb ? (n - J * tb) : tb);
            int64_t rp, rn, cp, cn;
            counts(I * tb, tb, rp, rn);
            counts(J * tb, bj, cp, cn);
            double same = (double)(rp * cp + rn * cn), opp = (double)(rp * cn + rn * cp);
            f += (2.0 * same + 4.0 * opp) * (double)tb;
        }
        return c * f;
    }
    // middle K blocks of block (I, I+D) split into bulk (I+L .. J-L) and edge (the rest)
    double gemm_bulk(int D, int L) const
    {
        const int nb = D - 2 * L + 1;
        return nb > 0 ? per_k_block(D) * nb : 0.0;
    }
    double gemm_edge(int D, int L) const
    {
        const int ne = D <= 1 ? 0 : (D - 1 < 2 * (L - 1) ? D - 1 : 2 * (L - 1));
        return ne > 0 ? per_k_block(D) * ne : 0.0;
    }
    double solve(int D) const
    {
        const int64_t nb = (n + tb - 1) / tb;
        double f = 0.0;
        for (int64_t I = 0; I + D < nb; ++I) {
            int64_t J = I + D;
            int bj = (int)((n - J * tb) < tb ? (n - J * tb) : tb);
            for (int i = 0; i < tb; ++i)
                for (int j = 0; j < bj; ++j) {
                    double w = (double)((tb - 1 - i) + j);
                    f += (s[I * tb + i] == s[J * tb + j] ? 2.0 : 4.0) * w;
                }
        }
        return c * f;
    }
    double diag() const
    {
        double f = 0.0;
        for (int64_t r0 = 0; r0 < n; r0 += tb) {
            int bt = (int)((n - r0) < tb ? (n - r0) : tb);
            for (int j = 0; j < bt; ++j)
                for (int i = 0; i < j; ++i)
                    f += (s[r0 + i] == s[r0 + j] ? 2.0 : 4.0) * (double)(j - i - 1);
        }
        return c * f;
    }
};

// One real blocked sweep (64 x 64 blocks): bulk products on a side stream,
// edge products and solves on the caller's stream.
struct RealSweep {
    const double *T;
    int64_t ldt;
    double *U;
    int64_t ldu;
    int64_t n;
    const int8_t *sgn;
    double *zbuf[kLookahead];   // bulk partials, by superdiagonal mod kLookahead
    double *ebuf;               // edge partials
    int64_t zslots;
    int max_splits;
    int tile;                   // 32 or 64
    const FlopCounter *flops;   // null unless timers are on
    std::vector<int> bulk_nm;   // bulk slices used per superdiagonal
};
hipError_t run_ph_real(RealSweep &w, hipStream_t st);
int64_t ph_real_edge_slots(int64_t n, int tb);
// Right-hand sides of block superdiagonal D (real, 64 x 64 blocks): nmid_split
// slices of the middle K blocks plus one slice for the diagonal-block terms,
// into Z[(tile * (nmid_split + 1) + slice) * 64 * 64 + i * 64 + j].
template <typename F>
hipError_t launch_wave_gemm(int tb, const F *T, int64_t ldt, const F *U, int64_t ldu, int64_t n,
                            const int8_t *sgn, int D, int ntiles, int edge, int nmid_split, int L,
                            F *Z, hipStream_t st);
int wave_gemm_mid_splits(int D, int L, int ntiles, int max_splits, int64_t zslots);
int wave_gemm_edge_slices(int D, int L);

// ---------------------------------------------------------------------------
// Persistent dataflow sweep (flow.hip): 32 x 32 blocks, one workgroup per block
// task, completion flags between tasks.
// ---------------------------------------------------------------------------
constexpr int kFlowTile = 32;
// A minority sign class of at most n / kStripDiv entries takes the residual's
// entries of differing signs from strips over its rows and columns.
constexpr int kStripDiv = 32;

// ---------------------------------------------------------------------------
// Projector form (proj.hip): the Parlett-Sylvester result for an ungrouped
// diagonal with at most kProjMaxMinorityReal (real T) or kProjMaxMinority
// (complex T) entries in its minority sign class.
// ---------------------------------------------------------------------------
constexpr int kProjMaxMinority = 64;
constexpr int kProjMaxMinorityReal = 512;
// Workspace of the form for order n and m minority entries (real: m up to
// kProjMaxMinorityReal; complex: kProjMaxMinority, whatever m).
size_t proj_workspace_bytes(int64_t n, int m, bool cplx);
// T, U column-major real; sgn the device sign vector; minority = its sign (+1/-1),
// m = its count.  Queues every launch on st.
// flops: algorithmic flops of the two substitutions, for the kernel timers.
// hsgn: the same signs on the host.
// herr: NULL, or host memory for the error word: then the call waits for the
// result and returns SIGNTRI_EHIP if a dependency wait of the persistent
// substitution kernel gave up.
// SIGNTRI_ENOTSUP when m is out of range or n too large for one resident grid.
// rcp_guard: some |t_ii| lies outside [2^-1020, 2^1019], where a reciprocal of
// t_ii - t_jj by the hardware estimate could leave the normal range.
int run_proj(const double *T, int64_t ldt, double *U, int64_t ldu, int64_t n, const int8_t *sgn,
             const int8_t *hsgn, int minority, int m, double flops, void *ws, hipStream_t st,
             int *herr, bool rcp_guard);
// Whether run_proj takes order n with m minority entries on the current device
// (its grid fits at once).
bool proj_fits(int64_t n, int m);
// The same for complex T (interleaved complex128).
int run_proj_c(const void *T, int64_t ldt, void *U, int64_t ldu, int64_t n, const int8_t *sgn,
               const int8_t *hsgn, int minority, int m, double flops, void *ws, hipStream_t st);
enum FlowKind { FLOW_MAIN = 0, FLOW_CORR = 1, FLOW_SYL = 2 };

// One real triangular system of a sweep; column-major device arrays.
//   MAIN: V = U (its diagonal blocks already computed), products of V and T.
//   CORR: V holds the residual on entry and the correction E on exit; C = U0.
//   SYL:  the unknown X = V(0:split, split:n), A = T(0:split, 0:split),
//         B = T(split:n, split:n), right-hand side rhs_scale * Rh(0:split, split:n)
//         (Rh = T for the Parlett-Sylvester equation, a residual for its correction).
template <typename F> struct FlowMat {
    const F *T;
    int64_t ldt;
    const F *C;
    int64_t ldc;
    F *V;
    int64_t ldv;
    const F *Rh;
    int64_t ldrh;
    const double *dg;    // FP64 diagonal of T (n entries)
    const int8_t *sgn;   // sign(Re t_ii) as +1 / -1 (n entries)
    int n;
    int split;           // SYL: order of T11
    int nbr, nbc;        // blocks in the row and column index spaces of the unknown
    int64_t flag0;       // this matrix's first completion flag (flags are I * nbc + J)
    double rhs_scale;    // SYL: 2 s
    int general;         // MAIN: a general function (Algorithm 1): every pair of entries by
                         // the element Parlett equation, V's diagonal blocks holding phi(T_II)
    int dense;           // MAIN, CORR: every 16 x 16 piece forms both accumulators
};
template <typename F> struct FlowArgs {
    FlowMat<F> m0;             // the matrix, when mats is null
    const FlowMat<F> *mats;    // per-matrix table (batched), or null
    const int2 *tasks;         // (matrix, I << 16 | J) in dependency order
    int ntasks;
    int *ctrl;                 // [0] ticket counter (zeroed before each sweep), [1] error
                               // word (zeroed once per run, so it keeps an earlier sweep's)
    int *flags;                // completion flags (zeroed before, or 1 for blocks not recomputed)
    int spin_limit;            // polls before a wait gives up and sets the error word
                               // (negative: the first wait gives up at once; testing)
    const int *live;           // if not null: the sweep runs only if *live != 0 (a refinement
                               // step that the device decided is needed)
    const int *ntasks_dev;     // if not null: the task count, at most ntasks, read on the
                               // device (a task list built on the device)
};
// C: complex entries (interleaved re, im).
template <typename F, int KIND, bool C>
hipError_t launch_flow(const FlowArgs<F> &a, int wgs_per_cu, hipStream_t st);
// Most workgroups per compute unit that fit, over the sweeps of one precision
// (wgs_per_cu above a kernel's own limit is clamped at launch).
int flow_max_wgs_per_cu(bool fp32, bool cplx);
int flow_default_wgs_per_cu(bool fp32, bool cplx);
hipError_t launch_fill_int(int *p, int64_t n, int v, hipStream_t st);
hipError_t launch_tasks_tri(int nb, int mat, int2 *out, hipStream_t st);
hipError_t launch_tasks_rect(int nbr, int nbc, int mat, int2 *out, hipStream_t st);
// (ntasks_dev: if not null, the count, at most ntasks, read on the device)
hipError_t launch_clear_task_flags(const int2 *tasks, int64_t ntasks, const int *ntasks_dev,
                                   const FlowMat<double> *mats, int *flags, hipStream_t st);

// Algorithmic flops of the launches of one call (Section 3 counting), for the
// opt-in kernel timers; all zero when the timers are off.
struct SweepFlops {
    double diag = 0, flow = 0, corr = 0, resid = 0, syl = 0;
};

// refine.hip: one real matrix of a reduced-precision computation.  The
// kernels take a table of these (blockIdx.z or the task's matrix index), or
// the single matrix m0 when the table pointer is null.
struct RefMat {
    const double *T;
    int64_t ldt;
    double *U;
    int64_t ldu;
    float *T32, *U32, *E32;    // FP32 copies of T and U0; residual / correction
    int64_t ld32;
    const int8_t *sgn;
    int n, split;              // split > 0: Sylvester form, X = U(0:split, split:n)
    int nbr, nbc;
    double two_s;              // Sylvester: 2 s
    int64_t f0;                // this matrix's first entry in the per-block arrays
    int64_t fr0;               // its first entry in the per-block-row arrays (nbr + 1 of them)
    unsigned long long *maxes; // max |t|, max |u0|, max |correction| (non-negative bits)
};
struct RefArgs {
    RefMat m0;
    const RefMat *mats;
    int nmat;
    const int *live;           // if not null: the kernels run only if *live != 0
};
hipError_t launch_to_f32(const RefArgs &a, int64_t nmax, bool cplx, hipStream_t st);
hipError_t launch_widen(const RefArgs &a, int64_t nmax, bool cplx, hipStream_t st);
hipError_t launch_add_correction(const RefArgs &a, int64_t nmax, bool cplx, hipStream_t st);
hipError_t launch_resid(const RefArgs &a, bool syl, bool cplx, const int2 *tasks, int ntasks,
                        double *norm2, hipStream_t st);
// Real substitution form on 128 x 128 tiles (matrix, a << 16 | b), a <= b; yonly:
// the entries of equal signs only (the others by launch_resid_strips, after it).
hipError_t launch_resid128(const RefArgs &a, const int2 *tiles, int ntiles, double *norm2,
                           hipStream_t st, bool yonly = false);
// The entries of differing signs of matrices with a small minority class: tasks
// (matrix, kind, group g: minority indices minl[16 g .. 16 g + 15], start of a
// 16-wide range); groups[g] = (matrix, 0, offset of its k-major copies in gbuf,
// low and high word); nmax: the largest order.
hipError_t launch_resid_strips(const RefArgs &a, const int4 *tasks, int ntasks, const int *minl,
                               const int4 *groups, int ngroups, int64_t nmax, double *gbuf,
                               double *norm2, hipStream_t st);

// The refinement's decisions on the device, so that the whole refinement is
// queued without a wait on the host (and can be captured in a graph).
// After step `step` (run only if *live_in): per block f of the task list,
// with a = sqrt(cur[f]) and aprev = sqrt(prev[f]) (rinit[f] = aprev at step 1):
// converged if a <= max(rounding floor, conv * rinit[f]) and not forced; stalled
// (sticky) if not converged and forced or a > stall * aprev; *live_out = 1 if
// some block is neither.
struct DecideArgs {
    const RefMat *mats;
    const int2 *tasks;         // the substitution blocks, then the Sylvester blocks
    int ntasks;
    const double *prev, *cur;  // squared residual norms before and after the step
    double *rinit;             // residual norm before the first step
    int8_t *ok, *hopeless;     // per block: converged; stalled
    const int *live_in;
    int *live_out;
    int step, nmat;
    double stall, conv;
    int64_t force;             // -1: every block forced to stall; k > 0 (one matrix): block k - 1
};
hipError_t launch_refine_decide(const DecideArgs &d, hipStream_t st);
// The FP64 recomputation's task lists: the blocks that did not converge and every
// block whose products read them (block (I, J) is read by (I', J') with I' <= I
// and J' >= J), in the order of the task lists, built on the device; counts in
// cnt[0] (substitution) and cnt[1] (Sylvester), per matrix in nfb.
struct ConeArgs {
    const RefMat *mats;
    const int2 *tasks;
    int nph, nps;              // the task list's two parts
    const int8_t *ok;
    int *rowmin;               // per block row (fr0 + I): the least J not converged there, and
                               // then over the rows below too
    int2 *out_ph, *out_ps;     // the recomputation's task lists
    int *cnt;                  // [2]
    int64_t *nfb;              // per matrix: blocks recomputed
};
hipError_t launch_refine_cone(const ConeArgs &c, int nmat, int64_t nrows, hipStream_t st);

// batch.hip: table-driven scan, output preparation and diagonal blocks.
struct ScanMat {
    const double *T;
    int64_t ldt;
    int64_t n;
    int8_t *sgn;
    double *dg;          // the diagonal (complex: re, im pairs)
    ScanResult *res;
    int cplx;            // complex entries (interleaved re, im)
};
struct PrepMat {
    const double *T;
    int64_t ldt;
    double *U;
    int64_t ldu;
    int64_t n;
    const int8_t *sgn;
    int kind;   // 0: zero the strict lower triangle; 1: diag(s I_p, -s I_{n-p}); 2: s I
    int64_t p;
    double s;
    const double *fd;  // a general function: phi(t_ii) (complex: re, im pairs); else null
};
hipError_t launch_scan_b(const ScanMat *mats, int nmat, hipStream_t st);
hipError_t launch_prepare_b(const PrepMat *mats, int nmat, int64_t nmax, bool cplx, hipStream_t st);
hipError_t launch_diag_b(const PrepMat *mats, const int2 *tasks, int ntasks, bool cplx,
                         hipStream_t st);

// sweep.hip: one real matrix of a run (a single call, or one matrix of a batch).
struct RealItem {
    const double *T;
    int64_t ldt;
    double *U;
    int64_t ldu;
    int64_t n;
    int path;             // SIGNTRI_PATH_*
    int64_t p;            // Parlett-Sylvester: order of the leading sign group
    int s;                // its sign (trivial path: the one sign)
    const int8_t *sgn;    // device signs and real diagonal
    const double *dg;     // (complex: interleaved re, im pairs)
    bool cplx;            // complex entries (interleaved re, im); the same for every item
    signtri_info *info;   // optional host output
    const double *fd = nullptr;  // a general function phi (path PH, FP64): phi(t_ii) on the
                                 // device (complex: re, im pairs); null for the sign
};
// Device and pinned-host bytes a run over these orders needs.
void run_sizes(const int64_t *ns, int nmat, bool mixed, bool cplx, size_t *dev_bytes,
               size_t *host_bytes);
// Run the sweeps of a set of real matrices: FP64, FP32, or FP32 with FP64
// refinement (mode), every phase one launch over all matrices.  The refinement
// decides on the device; with finish, the call then waits and reads its
// summary (refine_finish); without, nothing waits on the host (graph capture),
// and the caller calls refine_finish after the work has been queued.
int run_real(std::vector<RealItem> &items, signtri_mode mode, const signtri_options *opts,
             void *dev_ws, void *host_ws, bool prof, const int8_t *const *host_signs,
             hipStream_t st, bool finish = true);
// The refinement's outcome: waits for st, fills the items' infos (steps run,
// correction size, blocks recomputed); SIGNTRI_EHIP if a dependency wait gave
// up, SIGNTRI_ENOCONV if blocks did not converge and options forbid the FP64
// recomputation.
int refine_finish(std::vector<RealItem> &items, const signtri_options *opts, void *dev_ws,
                  void *host_ws, hipStream_t st);
// Refinement steps at most (options beyond it are rejected).
constexpr int kMaxRefineSteps = 64;
// Fixed buffers of the no-allocation entry point (device scratch and host
// staging) in place of the library-owned workspace.
struct NoAllocBuffers {
    void *dev;
    size_t dev_bytes;
    void *host;
    size_t host_bytes;
};
// signtri() with, when na is given, na's buffers instead of any allocation
// (FP64, column-major, AUTO, default options only: the dataflow sweeps or the
// projector form; SIGNTRI_ETOOBIG when the buffers are too small).
int signtri_run(const void *T, int64_t ldt, void *U, int64_t ldu, int64_t n, signtri_dtype dtype,
                signtri_layout layout, signtri_mode mode, signtri_algo algo, void *workspace,
                size_t ws_bytes, void *stream, const signtri_options *opts, signtri_info *info,
                const NoAllocBuffers *na);
// Device and host bytes signtri_run() takes from NoAllocBuffers for order n.
size_t noalloc_device_bytes(int64_t n, signtri_dtype dtype);
size_t noalloc_host_bytes(int64_t n, signtri_dtype dtype);

// Polls a dependency wait of the persistent kernels (the dataflow sweeps, the
// projector form's substitutions) makes before it gives up and sets the error word.  Testing hook: SIGNTRI_DEBUG_SPIN_LIMIT=-1 makes the first
// wait of every sweep give up at once (the kernels still run to their end, on
// whatever the operands hold), so that the host's check of the error word can be
// exercised.
int flow_spin_limit();
// Wait for a run and report whether a dependency wait hit its safety bound.
int sweep_error(void *dev_ws, const int64_t *ns, int nmat, bool mixed, bool cplx, void *host_ws,
                hipStream_t st, int *err);

// Diagonal 32 x 32 blocks of a real U in FP64 (Algorithm 3 per block).
hipError_t launch_diag_blocks(const double *T, int64_t ldt, double *U, int64_t ldu, int64_t n,
                              const int8_t *sgn, hipStream_t st);
// U = diag(s I_p, -s I_{n-p}), zeros elsewhere (real).
hipError_t launch_fill_split_identity(double *U, int64_t ldu, int64_t n, int64_t p, double s,
                                      hipStream_t st);

// block size used for a request (0 = default), and bulk partial-sum slots
int ph_tile_size(bool cplx, int requested);

// The autotuner's recorded choice for (dtype, mode, path, size class of n).
bool tune_find(signtri_dtype dtype, signtri_mode mode, int path, int64_t n,
               signtri_tune_entry *out);
int64_t ph_zslots(int64_t n, int tb);
hipError_t run_ph_fp64(const PhArgs &a, bool cplx, hipStream_t st);

}  // namespace sgt
