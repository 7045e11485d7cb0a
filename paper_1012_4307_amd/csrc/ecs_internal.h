// ecs_internal.h -- device data types and kernel launchers shared by the
// HIP translation units of the library (not part of the public ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecs {

// Interleaved complex number; 16 B (FP64) or 8 B (FP32), naturally aligned so
// a node is one 128-bit / 64-bit vector load.
template <typename R>
struct alignas(2 * sizeof(R)) cplx {
  R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cplx<R> mk(R re, R im) {
  cplx<R> z;
  z.re = re;
  z.im = im;
  return z;
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return mk<R>(a.re + b.re, a.im + b.im); }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return mk<R>(a.re - b.re, a.im - b.im); }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return mk<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator*(R s, cplx<R> a) { return mk<R>(s * a.re, s * a.im); }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> conjg(cplx<R> a) { return mk<R>(a.re, -a.im); }
template <typename R>
__host__ __device__ __forceinline__ R abs2(cplx<R> a) { return a.re * a.re + a.im * a.im; }
// a / b = a conj(b) / |b|^2
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cdiv(cplx<R> a, cplx<R> b) {
  R inv = R(1) / abs2(b);
  return inv * (a * conjg(b));
}
template <typename D, typename S>
__host__ __device__ __forceinline__ cplx<D> cvt(cplx<S> a) { return mk<D>(D(a.re), D(a.im)); }

// One level of the hierarchy as seen by a kernel.  The operator is
//   (M u)_p = sum_a [ cm_a(i_a) (u_p - u_{p - s_a}) + cp_a(i_a) (u_p - u_{p + s_a}) ]
//             + (beta k2_p + c) u_p
// with cm/cp the second-difference weights of Sec. 3.2 already multiplied by
// the operator's Laplacian factor alpha.  n2 == 1 in 2D.
template <typename R>
struct Grid {
  int n0, n1, n2;
  const cplx<R> *cm0, *cp0, *cm1, *cp1, *cm2, *cp2;
  const R *k2;
  cplx<R> beta, c;
};

// Grid rows through buffer resources.  One wave-uniform resource covers the
// rows [j_lo, j_hi) of an n0-wide array that a block may touch; a lane adds
// the byte offset of its column (fixed for the kernel) to the uniform offset
// of the row.  An offset at or beyond the resource's size reads 0 and drops a
// store (range-checked buffer access, no fault): rows outside the window and
// lanes outside the grid (column offset 2^31) need neither branches nor
// per-row address arithmetic.  Windows stay below 2^31 bytes.
constexpr uint32_t kOutside = 0x80000000u;   // column offset of a lane outside the grid
constexpr int kRsrcWord3 = 0x00020000;       // buffer resource word 3 for gfx9-family raw access

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const T *base, int j_lo, int j_hi, int n0) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)(base + (int64_t)j_lo * n0), 0,
                                           j_hi > j_lo ? (j_hi - j_lo) * n0 * (int)sizeof(T) : 0, kRsrcWord3);
}
template <typename T>
__device__ __forceinline__ uint32_t col_off(bool in, int i) {
  return in ? (uint32_t)i * (uint32_t)sizeof(T) : kOutside;
}
// byte offset of row q of the window (q < 0 wraps far outside)
template <typename T>
__device__ __forceinline__ uint32_t row_off(int q, int n0) {
  return (uint32_t)(q * n0 * (int)sizeof(T));
}
// Loaded values are bit-cast as a whole: with this compiler, indexing the
// elements of the vector the load builtins return narrows the access to its
// first dword.
__device__ __forceinline__ cplx<float> ld_c(__amdgpu_buffer_rsrc_t r, uint32_t off, cplx<float>) {
  return __builtin_bit_cast(cplx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ cplx<double> ld_c(__amdgpu_buffer_rsrc_t r, uint32_t off, cplx<double>) {
  return __builtin_bit_cast(cplx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ float ld_r(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double ld_r(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void st_c(__amdgpu_buffer_rsrc_t r, uint32_t off, cplx<float> v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, off,
                                        0, 0);
}
__device__ __forceinline__ void st_c(__amdgpu_buffer_rsrc_t r, uint32_t off, cplx<double> v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r, off,
                                         0, 0);
}

// Several right-hand sides of one system per launch (the batched solve): row
// y of the launch grid works on right-hand side slot[y] (rows = count).  The
// copies of a per-right-hand-side array of a level lie rhs_stride(nodes)
// elements apart; per-right-hand-side scalars are consecutive structs and
// reduction partials kRhsPartials entries apart.  A single solve launches
// one row with slot 0, so no pointer moves.
constexpr int kMaxRhs = 8;
constexpr int kRhsPartials = 8192;
struct RhsSet {
  int count;
  int slot[kMaxRhs];
};
__host__ __device__ __forceinline__ int64_t rhs_stride(int64_t nodes) { return (nodes + 63) & ~int64_t(63); }
__device__ __forceinline__ int64_t rhs_index(const RhsSet &rs) { return rs.slot[blockIdx.y]; }
inline RhsSet one_rhs() {
  RhsSet r{};
  r.count = 1;
  return r;
}
// launches for a map other than slot 0 alone use the kernels' multi-right-
// hand-side instantiations (template flag MR); single launches use the others,
// which never read the map
inline bool multi_rhs(const RhsSet &rs) { return rs.count > 1 || rs.slot[0] != 0; }

// XCD-aware tile order.  Workgroups are handed to the 8 XCDs of the chip in
// round-robin order of their linear index, and each XCD has its own L2.  A 1D
// launch of `padded` (a multiple of 8) blocks is mapped so that XCD x owns the
// contiguous tile range [x * padded/8, (x+1) * padded/8): neighbouring tiles,
// which share halo rows, are cached by the same L2.  Returns -1 for padding.
constexpr int kXcds = 8;
__host__ __device__ __forceinline__ int xcd_padded(int tiles) { return (tiles + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ int xcd_tile(int tiles) {
  const int padded = gridDim.x;
  const int b = blockIdx.x;
  const int t = (b % kXcds) * (padded / kXcds) + b / kXcds;
  return t < tiles ? t : -1;
}

// Kernel timing.  When a timed scope has armed these events, the next launch
// made through launch_k() records the kernel's own begin and end timestamps
// into them (hipExtLaunchKernelGGL) and disarms them, so a timed duration is
// the kernel's execution alone, without the dispatch latency that events
// recorded on the stream around the launch would add.
struct KernelEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local KernelEvents g_kernel_events;

template <typename... Args, typename F = void (*)(Args...)>
inline void launch_k(F kernel, const dim3 &grid, const dim3 &block, uint32_t shmem, hipStream_t s, Args... args) {
  KernelEvents &e = g_kernel_events;
  if (e.start) {
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, e.start, e.stop, 0, args...);
    e.start = e.stop = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
  }
}

// ---------------------------------------------------------------- launchers
// Multigrid components (kernels_mg.hip); R = double or float.
template <typename R, typename RI, typename RO>
void launch_apply(const Grid<R> &g, const cplx<RI> *x, cplx<RO> *y, hipStream_t s);
template <typename R>
void launch_residual(const Grid<R> &g, const cplx<R> *b, const cplx<R> *u, cplx<R> *r, hipStream_t s);
template <typename R>
void launch_jacobi(const Grid<R> &g, const cplx<R> *b, const cplx<R> *u, cplx<R> *out, R omega, bool zero_guess,
                   hipStream_t s);
template <typename R>
void launch_rb_colour(const Grid<R> &g, const cplx<R> *b, cplx<R> *u, R omega, int colour, bool zero_guess,
                      hipStream_t s);
template <typename R>
void launch_restrict(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *rf, cplx<R> *rc, hipStream_t s);
template <typename R>
void launch_residual_restrict(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, const cplx<R> *u,
                              cplx<R> *rc, hipStream_t s);
template <typename R>
void launch_prolong_add(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *ec, cplx<R> *u, hipStream_t s);
// u_out = u_in + P ec on the fine interior, 0 on its boundary (out of place)
template <typename R>
void launch_prolong_to(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *ec, const cplx<R> *u_in,
                       cplx<R> *u_out, hipStream_t s);
// 2D: out = one omega-Jacobi sweep of (u + P ec), out of place
template <typename R>
void launch_prolong_jacobi(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *ec, const cplx<R> *b,
                           const cplx<R> *u, cplx<R> *out, R omega, hipStream_t s);
template <typename R>
void launch_coarse_solve(int nunk, const cplx<R> *minv, const int *unk, int n0, int n1, int n2, const cplx<R> *b,
                         cplx<R> *x, hipStream_t s, const RhsSet &rs = one_rhs());
// fused V(1,1) red-black kernels (2D): zero-guess pre-sweep + residual + FW
// (the pre-smoothed iterate is not stored), and the pre-sweep recomputed from
// b + prolongation + correction + post-sweep into u_out
// (rows: tile height, see ecs_tuning)
template <typename R>
void launch_down_rb(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, cplx<R> *rc, R omega, int rows,
                    hipStream_t s, const RhsSet &rs = one_rhs());
// The down kernel can form its right-hand side while staging it, from the
// vectors of a Bi-CGSTAB step: kDownSrcP b = r + beta (p - omega v),
// kDownSrcS b = r - alpha v (the step's scalars read from S), each with the
// expression of the separate update kernels, so the values are the same.  The
// formed vector is stored at every node of the grid (out must not alias r, p
// or v: neighbouring blocks read them as their halo).
struct BicgScalars;
enum { kDownSrcB = 0, kDownSrcP = 1, kDownSrcS = 2 };
template <typename R>
struct DownSrc {
  int mode;                    // kDownSrcP or kDownSrcS
  const cplx<R> *r, *p, *v;    // p unused for kDownSrcS
  cplx<R> *out;
  const BicgScalars *S;
};
template <typename R>
void launch_down_rb_src(const Grid<R> &fine, const Grid<R> &coarse, const DownSrc<R> &src, cplx<R> *rc, R omega,
                        int rows, hipStream_t s);
template <typename R>
void launch_up_rb(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, const cplx<R> *ec, cplx<R> *u_out,
                  R omega, int rows, hipStream_t s, const RhsSet &rs = one_rhs());
// two levels of the fused cycle in one kernel (small levels): down over
// levels l, l+1 (writes u_l, u_{l+1}, b_{l+1} and b_{l+2}); up over levels
// l+1, l (reads the correction u_{l+2}, writes u_l)
template <typename R>
void launch_down2_rb(const Grid<R> &f, const Grid<R> &m, const Grid<R> &c, const cplx<R> *b, cplx<R> *t_f,
                     cplx<R> *b_m, cplx<R> *t_m, cplx<R> *rc, R omega, hipStream_t s, const RhsSet &rs = one_rhs());
template <typename R>
void launch_up2_rb(const Grid<R> &f, const Grid<R> &m, const Grid<R> &c, const cplx<R> *b_f, const cplx<R> *t_f,
                   const cplx<R> *b_m, const cplx<R> *t_m, const cplx<R> *ec, cplx<R> *u_out, R omega,
                   hipStream_t s, const RhsSet &rs = one_rhs());
// the coarsest levels of a 2D V(1,1) red-black cycle in one workgroup, every
// level vector resident in LDS: levels with at most kTailNodes nodes per axis,
// at least two of them (the last is the coarsest, solved densely), kTailCap
// nodes in all
constexpr int kTailMaxLevels = 8;
constexpr int kTailNodes = 33;
constexpr int kTailCap = 1536;
constexpr int kTailMinv = 2401;  // coarsest inverse entries staged in LDS (49 unknowns)
// FP32 cycles also have a wide tail: levels of up to kTailWideNodes nodes per
// axis, kTailWideCap nodes in all (a 65^2 level down to a 9^2 coarsest: 5684),
// with at most kTailWideWeights 1D weights per axis over its levels
constexpr int kTailWideNodes = 65;
constexpr int kTailWideCap = 5696;
constexpr int kTailWideWeights = 132;
template <typename R>
struct TailArgs {
  int nl;                            // levels in the tail, the last one the coarsest
  int noff[kTailMaxLevels + 1];      // node offsets of the levels in the LDS vectors
  int poff[kTailMaxLevels + 1];      // the same, each level padded to a multiple of 64 nodes
  int woff[kTailMaxLevels + 1];      // offsets of the levels' 1D weights
  Grid<R> g[kTailMaxLevels];
  const cplx<R> *b0;                 // right-hand side of the tail's first level
  cplx<R> *u0;                       // its result
  const cplx<R> *minvT;              // coarsest inverse, transposed
  int nunk;                          // interior nodes of the coarsest level, row-major
  int tpr;                           // threads per row of the dense solve (power of 2, <= 64)
  R omega;
};
template <typename R>
void launch_tail(const TailArgs<R> &a, hipStream_t s, const RhsSet &rs = one_rhs());

// The coarse end of a general cycle (any gamma_f, gamma_c, nu1, nu2,
// omega-Jacobi or red-black) in one workgroup, driven by a schedule that the
// host unrolls from Algorithm 1.  One 32-bit word per operation:
//   bits 0-3 code, 4-7 level k (0 = the tail's first level), 8 zero guess,
//   9 f0, 10 f1 (buffer / colour selectors, per code):
//   kSchedJacobi  u[f1] <- one omega-Jacobi sweep of u[f0] (zero guess: of 0)
//   kSchedRB      one colour f1 of a red-black sweep, in place on u[f0]
//   kSchedResid   b_{k+1} <- FW (b_k - M_k u[f0]_k)   (uses u[!f0]_k as scratch)
//   kSchedCoarse  u[f0]_k <- M_k^{-1} b_k              (k: the coarsest level)
//   kSchedProlong u[f0]_k += P u[f1]_{k+1}
//   kSchedZero    u[f0]_k <- 0
//   kSchedEnd     the tail's result is u[f0]_0
enum : uint32_t { kSchedEnd = 0, kSchedJacobi = 1, kSchedRB = 2, kSchedResid = 3, kSchedCoarse = 4,
                  kSchedProlong = 5, kSchedZero = 6 };
constexpr int kSchedPack = kTailCap + 512;  // packed weights + inverse diagonals of the tail levels
constexpr int kSchedProgCap = 4096;         // operations per schedule
template <typename R>
struct SchedArgs {
  int nl;                             // levels in the tail, the last one the coarsest
  int noff[kTailMaxLevels + 1];       // node offsets of the levels in the LDS vectors
  int pko[kTailMaxLevels + 1];        // offsets of the levels in the pack
  int n0[kTailMaxLevels], n1[kTailMaxLevels];
  const cplx<R> *pack;                // per level: alpha a-, alpha a+ (x), the same (y), 1 / diag(M)
  int pack_len;
  const cplx<R> *minvT;               // coarsest inverse, transposed
  int nunk, tpr;                      // coarsest interior nodes; threads per row of the dense solve
  const cplx<R> *b_in;                // right-hand side of the first level
  const cplx<R> *u_in;                // its initial iterate, or null for a zero guess
  cplx<R> *u_out;                     // its result (may alias u_in)
  const uint32_t *prog;
  int prog_len;
  R omega;
};
template <typename R>
void launch_sched_tail(const SchedArgs<R> &a, hipStream_t s);
template <typename R>
void launch_inject_k2(int n0, int n1, int n2, const double *k2_fine, int f0, int f1, R *k2_coarse, hipStream_t s);

}  // namespace ecs
