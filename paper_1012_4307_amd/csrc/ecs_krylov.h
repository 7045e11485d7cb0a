// ecs_krylov.h -- device-resident Krylov scalars and the launchers of the
// vector / reduction kernels (kernels_blas.hip).  Internal to the library.
#pragma once

#include "ecs_internal.h"

namespace ecs {

constexpr int kMaxRestart = 64;
// reduction kernels use at most this many blocks (partial buffers are sized for it)
constexpr int kRedBlocks = 2048;
// steps of the nested Bi-CGSTAB whose preconditioned directions are kept for
// the deferred x update (a longer inner run updates x every kDeferSteps steps)
constexpr int kDeferSteps = 24;

// Scalars of one GMRES / FGMRES solve, kept in device memory.
struct GmresScalars {
  cplx<double> nrm2;                                   // last reduced squared norm (.re)
  double bnorm;                                        // ||b||
  double inv;                                          // 1 / (norm of the newest basis vector)
  double est;                                          // |g_{j+1}| / ||b||  (Givens estimate)
  double resid_true;                                   // true residual / ||b|| at a restart
  int bad, happy;
  int reorth;                                          // the second Gram-Schmidt pass of this step runs
  int reorth_count;                                    // second passes run in this solve
  cplx<double> one;                                    // constant 1 (single-column updates)
  cplx<double> g[kMaxRestart + 1];
  cplx<double> cs[kMaxRestart], sn[kMaxRestart];
  cplx<double> y[kMaxRestart];
  cplx<double> h2[kMaxRestart + 1];                    // second Gram-Schmidt pass
  cplx<double> d2[2 * kMaxRestart + 2];                // products of the delayed second pass
  cplx<double> H[(kMaxRestart + 1) * kMaxRestart];     // column-major Hessenberg, ld = m+1
};

// Scalars of one Bi-CGSTAB solve.
struct BicgScalars {
  cplx<double> rho, alpha, omega, beta;
  double rnorm2, bnorm, est;
  int bad;
  int breakdowns;  // restarts (kBicgInit) that found the previous run ended by a bad scalar
};

enum { kBicgAlpha = 1, kBicgOmega = 2, kBicgInit = 4, kBicgNormRho = 5 };

int reduction_blocks(int64_t n);

// The Arnoldi kernels take an optional gate: with gate != null they do
// nothing unless *gate != 0 (a second Gram-Schmidt pass decided on the device).
// multi-dot partials: partials[c][block] = block's share of sum_p conj(V_c[p]) w[p]
template <typename RA, typename RB>
void launch_mdot_partial(const cplx<RA> *V, int64_t ldv, int ncols, const cplx<RB> *w, int64_t n,
                         cplx<double> *partials, hipStream_t s, const int *gate = nullptr);
// out[c] = fixed-order sum of partials[c][*] (block count derived from n)
void launch_reduce_cols(const cplx<double> *partials, int64_t n, int ncols, cplx<double> *out, hipStream_t s,
                        const int *gate = nullptr);
// w <- w - sum_c V_c h_c ; partials[block] = block's share of ||w||^2
void launch_mupdate_partial(const cplx<double> *V, int64_t ldv, int ncols, const cplx<double> *h, cplx<double> *w,
                            int64_t n, cplx<double> *partials, hipStream_t s, const int *gate = nullptr);
// delayed second pass (DCGS2): partials of [V_0..V_{ncols-1}, x]^H x and
// [V_0..V_{ncols-1}, x]^H w (2 ncols + 2 columns, layout in kernels_blas.hip)
void launch_mdot2_partial(const cplx<double> *V, int64_t ldv, int ncols, const cplx<double> *x,
                          const cplx<double> *w, int64_t n, cplx<double> *partials, hipStream_t s);
// x's second pass and w's first from the reduced products d; partials of
// ||w||^2; hcol[0..ncols] = w's Hessenberg column
void launch_mupdate2_partial(const cplx<double> *V, int64_t ldv, int ncols, const cplx<double> *d, cplx<double> *x,
                             cplx<double> *w, int64_t n, cplx<double> *partials, cplx<double> *hcol, hipStream_t s);
// S->reorth = (||w'||^2 = S->nrm2 < eta2 ||w||^2 = H(j+1, j)); counts it
void launch_reorth_gate(GmresScalars *S, int j, int m, double eta2, hipStream_t s);
template <typename R>
void launch_nrm2sq(const cplx<R> *x, int64_t n, cplx<double> *partials, cplx<double> *out, hipStream_t s);
template <typename RZ>
void launch_lincomb(const cplx<RZ> *Z, int64_t ldz, int ncols, const cplx<double> *y, cplx<double> *x, int64_t n,
                    hipStream_t s);
void launch_scale_dev(cplx<double> *x, int64_t n, const double *scal, hipStream_t s);
void launch_gmres_start(GmresScalars *S, int m, hipStream_t s);
void launch_gmres_givens(GmresScalars *S, int j, int m, hipStream_t s);
void launch_gmres_backsolve(GmresScalars *S, int k, int m, hipStream_t s);
void launch_add_h2(GmresScalars *S, int j, int m, hipStream_t s, const int *gate = nullptr);

template <typename R>
void launch_pairdot(const cplx<R> *x0, const cplx<R> *y0, const cplx<R> *x1, const cplx<R> *y1, int npairs, int64_t n,
                    cplx<double> *partials, BicgScalars *S, int mode, hipStream_t s);
// With an RhsSet (the batched solve) the vectors of slot q start q
// rhs_stride(n) elements in, the scalars at S + q and the partials
// q kRhsPartials entries in.
template <typename R>
void launch_bicg_p(cplx<R> *p, const cplx<R> *r, const cplx<R> *v, int64_t n, const BicgScalars *S, hipStream_t s,
                   const RhsSet &rs = one_rhs());
template <typename R>
void launch_bicg_s(cplx<R> *sv, const cplx<R> *r, const cplx<R> *v, int64_t n, const BicgScalars *S, hipStream_t s,
                   const RhsSet &rs = one_rhs());
// x += alpha ph + omega sh; r = s - omega t; then ||r||^2 and (r^, r) reduce
// (fixed-order second stage) into est and the next step's beta
template <typename R, typename RZ>
void launch_bicg_xr(cplx<R> *x, const cplx<RZ> *ph, const cplx<RZ> *sh, cplx<R> *r, const cplx<R> *sv,
                    const cplx<R> *t, const cplx<R> *rh, int64_t n, cplx<double> *partials, BicgScalars *S,
                    hipStream_t s, const RhsSet &rs = one_rhs());
// The nested Bi-CGSTAB with its x update deferred: r = s - omega t, the
// same reductions as launch_bicg_xr, and (alpha, omega) of the step stored at
// coef[0..1]; later x += sum_i alpha_i p^_i + omega_i s^_i over `count`
// stored steps (ld elements apart), in step order, each step the one-step
// update's expression.
template <typename R>
void launch_bicg_r(cplx<R> *r, const cplx<R> *sv, const cplx<R> *t, const cplx<R> *rh, int64_t n,
                   cplx<double> *partials, BicgScalars *S, cplx<double> *coef, hipStream_t s);
template <typename R>
void launch_bicg_xdefer(cplx<R> *x, const cplx<R> *ph, const cplx<R> *sh, int64_t ld, int count,
                        const cplx<double> *coef, int64_t n, hipStream_t s);
// y = A x with a fused dot product: kBicgAlpha -> (d0, y) gives alpha;
// kBicgOmega -> (y, d0) and (y, y) give omega (multigrid side, kernels_mg.hip)
void launch_bicg_final(const cplx<double> *partials, int nblocks, int npairs, BicgScalars *S, int mode,
                       hipStream_t s, const RhsSet &rs = one_rhs());
template <typename R, typename RI>
void launch_apply_dot(const Grid<R> &g, const cplx<RI> *x, cplx<R> *y, const cplx<R> *d0, int mode,
                      cplx<double> *partials, BicgScalars *S, hipStream_t s, const RhsSet &rs = one_rhs());

template <typename RI, typename RO>
void launch_cast(const cplx<RI> *x, cplx<RO> *y, int64_t n, hipStream_t s, const RhsSet &rs = one_rhs());
void launch_cast_real(const double *x, float *y, int64_t n, hipStream_t s);
// FP32 -> FP64 real array (exact)
void launch_widen_real(const float *x, double *y, int64_t n, hipStream_t s);
template <typename R>
void launch_zero(cplx<R> *x, int64_t n, hipStream_t s);
void launch_scale_w(int n0, int n1, int n2, const cplx<double> *w0, const cplx<double> *w1, const cplx<double> *w2,
                    const cplx<double> *x, cplx<double> *y, bool inverse, hipStream_t s);
void launch_mask_boundary(int n0, int n1, int n2, const cplx<double> *x, cplx<double> *y, hipStream_t s);
void launch_grad_k2(const cplx<double> *lam, const cplx<double> *u, double *g, int64_t n, hipStream_t s);
// coupled block system (nb <= kMaxBlocks): y_i -= sum_{j != i} k2c[i nb + j] x_j,
// then y_i = b_i - y_i when b is given
constexpr int kMaxBlocks = 8;
void launch_couple(int nb, int64_t nn, const double *k2c, const cplx<double> *x, cplx<double> *y,
                   const cplx<double> *b, hipStream_t s);
void launch_max_real(const double *x, int64_t n, double *partials, double *out, hipStream_t s);
void launch_copy_bytes(const void *src, void *dst, size_t bytes, hipStream_t s);
// a kernel that does nothing (timing calibration)
void launch_empty(hipStream_t s);

}  // namespace ecs
