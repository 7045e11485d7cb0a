// kernels_blas.hip -- Krylov building blocks of the outer solve (Sec. 5 of
// bin Zubair, Reps, Vanroose: right-preconditioned Bi-CGSTAB; GMRES and
// restarted / flexible GMRES).  All Krylov scalars stay in device memory: dot
// products reduce in two fixed-order stages (per-block partials, then one
// block per column), so results are bitwise reproducible run to run, and the
// Givens least-squares update and the Bi-CGSTAB scalar recurrences run in
// single-thread kernels right behind their reductions.  The host only reads a
// residual estimate per iteration.
#include "ecs_reduce.h"

namespace ecs {

namespace {

__global__ void k_empty() {}

constexpr int BS = kRedThreads;

inline int red_blocks(int64_t n) {
  int64_t b = (n + BS * 4 - 1) / (BS * 4);
  if (b > kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

// ----------------------------------------------------------- multi-dot
// out[c] = sum_p conj(V_c[p]) w[p], c < ncols.  A block walks tiles of
// BS * EPT nodes; each thread keeps its EPT entries of w in registers (w is
// read once) and treats the columns in groups of CG, so CG * EPT independent
// loads are in flight per thread.  Each column's tile sum is wave-reduced and
// lane 0 adds it to the wave's LDS accumulator; fixed order throughout, so
// the result is bitwise reproducible.
constexpr int EPT = 4;
constexpr int CG = 4;

template <typename RA, typename RB>
__global__ __launch_bounds__(BS) void k_mdot(const cplx<RA> *__restrict__ V, int64_t ldv, int ncols,
                                             const cplx<RB> *__restrict__ w, int64_t n, cplx<double> *partials,
                                             const int *gate) {
  if (gate && *gate == 0) return;  // a second Gram-Schmidt pass that is not needed
  constexpr int LDA = kMaxRestart + 2;
  __shared__ cplx<double> acc[BS / 64][LDA];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = threadIdx.x; c < (BS / 64) * LDA; c += BS) acc[c / LDA][c % LDA] = mk<double>(0, 0);
  __syncthreads();
  const int64_t tile = (int64_t)BS * EPT;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile) {
    cplx<double> wv[EPT];
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int64_t p = base + e * BS + threadIdx.x;
      wv[e] = p < n ? cvt<double>(w[p]) : mk<double>(0, 0);
    }
    for (int c0 = 0; c0 < ncols; c0 += CG) {
      cplx<double> sg[CG];
#pragma unroll
      for (int g = 0; g < CG; g++) {
        sg[g] = mk<double>(0, 0);
        if (c0 + g < ncols) {
          const cplx<RA> *vc = V + (int64_t)(c0 + g) * ldv;
#pragma unroll
          for (int e = 0; e < EPT; e++) {
            const int64_t p = base + e * BS + threadIdx.x;
            if (p < n) sg[g] = sg[g] + conjg(cvt<double>(vc[p])) * wv[e];
          }
        }
      }
#pragma unroll
      for (int g = 0; g < CG; g++) {
        if (c0 + g < ncols) {
          double re = wave_sum(sg[g].re), im = wave_sum(sg[g].im);
          if (lane == 0) acc[wid][c0 + g] = acc[wid][c0 + g] + mk<double>(re, im);
        }
      }
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncols; c += BS) {
    cplx<double> t = mk<double>(0, 0);
    for (int q = 0; q < BS / 64; q++) t = t + acc[q][c];
    partials[(int64_t)c * gridDim.x + blockIdx.x] = t;
  }
}

// out[c] = sum over blocks of partials[c][block] (fixed order); one block per
// column.
__global__ __launch_bounds__(BS) void k_reduce_cols(const cplx<double> *__restrict__ partials, int nblocks,
                                                    cplx<double> *__restrict__ out, const int *gate) {
  if (gate && *gate == 0) return;
  __shared__ cplx<double> lds[BS / 64];
  const int c = blockIdx.x;
  cplx<double> s = strided_sum(partials + (int64_t)c * nblocks, nblocks);
  s = block_sum(s, lds);
  if (threadIdx.x == 0) out[c] = s;
}

// w <- w - sum_c V_c h_c, and per-block partials of ||w||^2 (in .re); same
// tiling as the multi-dot
__global__ __launch_bounds__(BS) void k_mupdate(const cplx<double> *__restrict__ V, int64_t ldv, int ncols,
                                                const cplx<double> *__restrict__ h, cplx<double> *__restrict__ w,
                                                int64_t n, cplx<double> *partials, const int *gate) {
  if (gate && *gate == 0) return;
  __shared__ cplx<double> hs[kMaxRestart + 2];
  __shared__ cplx<double> lds[BS / 64];
  for (int c = threadIdx.x; c < ncols; c += BS) hs[c] = h[c];
  __syncthreads();
  double nrm = 0;
  const int64_t tile = (int64_t)BS * EPT;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile) {
    cplx<double> wv[EPT];
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int64_t p = base + e * BS + threadIdx.x;
      wv[e] = p < n ? w[p] : mk<double>(0, 0);
    }
    for (int c0 = 0; c0 < ncols; c0 += CG) {
#pragma unroll
      for (int g = 0; g < CG; g++) {
        if (c0 + g < ncols) {
          const cplx<double> *vc = V + (int64_t)(c0 + g) * ldv;
          const cplx<double> hc = hs[c0 + g];
#pragma unroll
          for (int e = 0; e < EPT; e++) {
            const int64_t p = base + e * BS + threadIdx.x;
            if (p < n) wv[e] = wv[e] - vc[p] * hc;
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int64_t p = base + e * BS + threadIdx.x;
      if (p < n) {
        w[p] = wv[e];
        nrm += abs2(wv[e]);
      }
    }
  }
  cplx<double> s = block_sum(mk<double>(nrm, 0), lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// ------------------------------------- delayed second pass (DCGS2)
// The newest basis vector x = v_j has had one Gram-Schmidt pass (and its
// normalisation) when the next direction w = A z_j arrives; its second pass
// is taken together with w's first: one multi-dot of the columns
// V_0..V_{ncols-1} and x itself against both x and w, then one update pass
// over the same columns for both vectors.
//   partial columns c < ncols:        sum conj(V_c) x      (s_c)
//                   c = ncols:        sum conj(x) x        (alpha)
//                   ncols + 1 + c:    sum conj(V_c) w      (g_c)
//                   2 ncols + 1:      sum conj(x) w        (beta)
// Same tiling and fixed summation order as the one-vector multi-dot.
__global__ __launch_bounds__(BS) void k_mdot2(const cplx<double> *__restrict__ V, int64_t ldv, int ncols,
                                              const cplx<double> *__restrict__ x, const cplx<double> *__restrict__ w,
                                              int64_t n, cplx<double> *partials) {
  constexpr int LDA = 2 * kMaxRestart + 2;
  __shared__ cplx<double> acc[BS / 64][LDA];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nout = 2 * ncols + 2;
  for (int c = threadIdx.x; c < (BS / 64) * LDA; c += BS) acc[c / LDA][c % LDA] = mk<double>(0, 0);
  __syncthreads();
  const int64_t tile = (int64_t)BS * EPT;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile) {
    cplx<double> xv[EPT], wv[EPT];
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int64_t p = base + e * BS + threadIdx.x;
      xv[e] = p < n ? x[p] : mk<double>(0, 0);
      wv[e] = p < n ? w[p] : mk<double>(0, 0);
    }
    for (int c0 = 0; c0 < ncols; c0 += CG) {
      cplx<double> sx[CG], sw[CG];
#pragma unroll
      for (int g = 0; g < CG; g++) {
        sx[g] = mk<double>(0, 0);
        sw[g] = mk<double>(0, 0);
        if (c0 + g < ncols) {
          const cplx<double> *vc = V + (int64_t)(c0 + g) * ldv;
#pragma unroll
          for (int e = 0; e < EPT; e++) {
            const int64_t p = base + e * BS + threadIdx.x;
            if (p < n) {
              const cplx<double> cv = conjg(vc[p]);
              sx[g] = sx[g] + cv * xv[e];
              sw[g] = sw[g] + cv * wv[e];
            }
          }
        }
      }
#pragma unroll
      for (int g = 0; g < CG; g++) {
        if (c0 + g < ncols) {
          double xr = wave_sum(sx[g].re), xi = wave_sum(sx[g].im);
          double wr = wave_sum(sw[g].re), wi = wave_sum(sw[g].im);
          if (lane == 0) {
            acc[wid][c0 + g] = acc[wid][c0 + g] + mk<double>(xr, xi);
            acc[wid][ncols + 1 + c0 + g] = acc[wid][ncols + 1 + c0 + g] + mk<double>(wr, wi);
          }
        }
      }
    }
    // the vector x as a column: alpha = (x, x), beta = (x, w)
    cplx<double> sa = mk<double>(0, 0), sb = mk<double>(0, 0);
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      sa = sa + conjg(xv[e]) * xv[e];
      sb = sb + conjg(xv[e]) * wv[e];
    }
    double ar = wave_sum(sa.re), br = wave_sum(sb.re), bi = wave_sum(sb.im);
    if (lane == 0) {
      acc[wid][ncols] = acc[wid][ncols] + mk<double>(ar, 0);
      acc[wid][2 * ncols + 1] = acc[wid][2 * ncols + 1] + mk<double>(br, bi);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < nout; c += BS) {
    cplx<double> t = mk<double>(0, 0);
    for (int q = 0; q < BS / 64; q++) t = t + acc[q][c];
    partials[(int64_t)c * gridDim.x + blockIdx.x] = t;
  }
}

// Coefficients of the delayed pass from the reduced products d (layout of
// k_mdot2) -- every block derives the same values in the same order:
//   nu = sqrt(alpha - sum |s_c|^2)     norm of x after its second pass
//   h  = (beta - sum conj(s_c) g_c) / nu = (x after the pass, w)
// With no earlier columns (the first step of a cycle, x = r / ||r|| exactly)
// nu = 1.  Should alpha - sum |s|^2 not be positive (x numerically inside the
// span of the basis) the second pass of x is skipped (s = 0, nu = 1).
// Coefficients stored in k[0] = (1 / nu, pass ? 1 : 0), k[1] = h.
__device__ inline void dcgs2_coef(const cplx<double> *d, int ncols, cplx<double> *k) {
  double ss = 0;
  cplx<double> sg = mk<double>(0, 0);
  for (int c = 0; c < ncols; c++) {
    ss += abs2(d[c]);
    sg = sg + conjg(d[c]) * d[ncols + 1 + c];
  }
  const double nu2 = d[ncols].re - ss;
  const bool pass = ncols > 0 && nu2 > 0 && !isinf(nu2);
  const double inv_nu = pass ? 1.0 / sqrt(nu2) : 1.0;
  k[0] = mk<double>(inv_nu, pass ? 1.0 : 0.0);
  k[1] = pass ? inv_nu * (d[2 * ncols + 1] - sg) : d[2 * ncols + 1];
}

// The update pass of the delayed step (ncols columns before x):
//   x <- (x - sum_c V_c s_c) / nu           (x's second pass; skipped for ncols = 0)
//   w <- w - sum_c V_c g_c - h x            (w's first pass against V and the new x)
// partials[block] = the block's share of ||w||^2; block 0 stores the
// Hessenberg column H(0..ncols, j) = (g_0, ..., g_{ncols-1}, h).
__global__ __launch_bounds__(BS) void k_mupdate2(const cplx<double> *__restrict__ V, int64_t ldv, int ncols,
                                                 const cplx<double> *__restrict__ d, cplx<double> *__restrict__ x,
                                                 cplx<double> *__restrict__ w, int64_t n, cplx<double> *partials,
                                                 cplx<double> *hcol) {
  __shared__ cplx<double> ss[kMaxRestart], gs[kMaxRestart];
  __shared__ cplx<double> lds[BS / 64];
  __shared__ cplx<double> kc[2];
  for (int c = threadIdx.x; c < ncols; c += BS) {
    ss[c] = d[c];
    gs[c] = d[ncols + 1 + c];
  }
  if (threadIdx.x == 0) dcgs2_coef(d, ncols, kc);
  __syncthreads();
  const double inv_nu = kc[0].re;
  const bool pass = kc[0].im != 0;
  const cplx<double> hx = kc[1];
  if (blockIdx.x == 0) {
    if ((int)threadIdx.x < ncols) hcol[threadIdx.x] = gs[threadIdx.x];
    else if ((int)threadIdx.x == ncols) hcol[ncols] = kc[1];
  }
  double nrm = 0;
  const int64_t tile = (int64_t)BS * EPT;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile) {
    cplx<double> xv[EPT], wv[EPT];
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int64_t p = base + e * BS + threadIdx.x;
      xv[e] = p < n ? x[p] : mk<double>(0, 0);
      wv[e] = p < n ? w[p] : mk<double>(0, 0);
    }
    for (int c0 = 0; c0 < ncols; c0 += CG) {
#pragma unroll
      for (int g = 0; g < CG; g++) {
        if (c0 + g < ncols) {
          const cplx<double> *vc = V + (int64_t)(c0 + g) * ldv;
          const cplx<double> sc = pass ? ss[c0 + g] : mk<double>(0, 0), gc = gs[c0 + g];
#pragma unroll
          for (int e = 0; e < EPT; e++) {
            const int64_t p = base + e * BS + threadIdx.x;
            if (p < n) {
              const cplx<double> v = vc[p];
              xv[e] = xv[e] - v * sc;
              wv[e] = wv[e] - v * gc;
            }
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int64_t p = base + e * BS + threadIdx.x;
      if (p < n) {
        const cplx<double> xn = inv_nu * xv[e];
        wv[e] = wv[e] - xn * hx;
        if (pass) x[p] = xn;
        w[p] = wv[e];
        nrm += abs2(wv[e]);
      }
    }
  }
  cplx<double> s = block_sum(mk<double>(nrm, 0), lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename R>
__global__ __launch_bounds__(BS) void k_nrm2sq(const cplx<R> *__restrict__ x, int64_t n, cplx<double> *partials) {
  __shared__ cplx<double> lds[BS / 64];
  double nrm = 0;
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS)
    nrm += abs2(cvt<double>(x[p]));
  cplx<double> s = block_sum(mk<double>(nrm, 0), lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// x[p] += sum_c Z_c[p] y_c  (Z in the preconditioner's precision)
template <typename RZ>
__global__ __launch_bounds__(BS) void k_lincomb(const cplx<RZ> *__restrict__ Z, int64_t ldz, int ncols,
                                                const cplx<double> *__restrict__ y, cplx<double> *__restrict__ x,
                                                int64_t n) {
  __shared__ cplx<double> ys[kMaxRestart + 2];
  for (int c = threadIdx.x; c < ncols; c += BS) ys[c] = y[c];
  __syncthreads();
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) {
    cplx<double> acc = x[p];
    for (int c = 0; c < ncols; c++) acc = acc + cvt<double>(Z[(int64_t)c * ldz + p]) * ys[c];
    x[p] = acc;
  }
}

// x *= *s  (s real, in device memory)
__global__ __launch_bounds__(BS) void k_scale_dev(cplx<double> *__restrict__ x, int64_t n,
                                                  const double *__restrict__ s) {
  const double f = *s;
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) x[p] = f * x[p];
}

// ------------------------------------------------------ GMRES scalars
// Start of a restart cycle: beta = sqrt(norm2) of the residual; g = beta e1;
// inv = 1/beta (the residual is scaled into v_0); est = beta / ||b||.
__global__ void k_gmres_start(GmresScalars *S, int m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double beta = sqrt(S->nrm2.re);
  for (int q = 0; q <= m; q++) S->g[q] = mk<double>(0, 0);
  S->g[0] = mk<double>(beta, 0);
  S->inv = beta > 0 ? 1.0 / beta : 0.0;
  S->est = beta / S->bnorm;
  S->resid_true = beta / S->bnorm;
  S->bad = !(beta == beta) || isinf(beta);
}

// Arnoldi step j: column j of the Hessenberg matrix holds h_{0..j,j} from the
// orthogonalisation; h_{j+1,j} = sqrt(norm2).  Apply the stored Givens
// rotations, form the new one, update g and the residual estimate |g_{j+1}|.
__global__ void k_gmres_givens(GmresScalars *S, int j, int m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  cplx<double> *h = S->H + (int64_t)j * (m + 1);
  double hn = sqrt(S->nrm2.re);
  h[j + 1] = mk<double>(hn, 0);
  S->inv = hn > 0 ? 1.0 / hn : 0.0;
  for (int i = 0; i < j; i++) {
    cplx<double> c = S->cs[i], s = S->sn[i];
    cplx<double> t = conjg(c) * h[i] + s * h[i + 1];
    h[i + 1] = (c * h[i + 1]) - (conjg(s) * h[i]);
    h[i] = t;
  }
  // new rotation zeroing h[j+1]: c = |a|/r (real), s = (a/|a|) conj(b) / r
  cplx<double> a = h[j], b = h[j + 1];
  double na = sqrt(abs2(a)), nb = sqrt(abs2(b));
  cplx<double> c, s;
  if (nb == 0) {
    c = mk<double>(1, 0); s = mk<double>(0, 0);
  } else if (na == 0) {
    c = mk<double>(0, 0); s = mk<double>(1, 0);
  } else {
    double r = sqrt(na * na + nb * nb);
    c = mk<double>(na / r, 0);
    s = (1.0 / (na * r)) * (a * conjg(b));
  }
  S->cs[j] = c;
  S->sn[j] = s;
  h[j] = conjg(c) * a + s * b;
  h[j + 1] = mk<double>(0, 0);
  cplx<double> gj = S->g[j];
  S->g[j] = conjg(c) * gj;
  S->g[j + 1] = mk<double>(0, 0) - conjg(s) * gj;
  S->est = sqrt(abs2(S->g[j + 1])) / S->bnorm;
  S->bad = !(S->est == S->est) || isinf(S->est);
  S->happy = hn == 0;
}

// y = R^{-1} g for the first k columns (upper triangular from the rotated H)
__global__ void k_gmres_backsolve(GmresScalars *S, int k, int m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int r = k - 1; r >= 0; r--) {
    cplx<double> s = S->g[r];
    for (int c = r + 1; c < k; c++) s = s - S->H[(int64_t)c * (m + 1) + r] * S->y[c];
    const cplx<double> d = S->H[(int64_t)r * (m + 1) + r];
    // a zero pivot only arises when the preconditioned vector vanished (w = 0);
    // that direction then carries no information and gets a zero coefficient
    S->y[r] = abs2(d) > 0 ? cdiv(s, d) : mk<double>(0, 0);
  }
}

// second Gram-Schmidt pass: H(:, j) += h2 (when the pass ran)
__global__ void k_add_h2(GmresScalars *S, int j, int m, const int *gate) {
  if (gate && *gate == 0) return;
  int q = threadIdx.x;
  if (q <= j) S->H[(int64_t)j * (m + 1) + q] = S->H[(int64_t)j * (m + 1) + q] + S->h2[q];
}

// Selective reorthogonalisation (the criterion of Daniel, Gragg, Kaufman and
// Stewart): after the first pass, ||w'||^2 is in S->nrm2 and ||w||^2 before it
// in H(j+1, j) (the multi-dot's extra column); a second pass runs when the
// projection removed so much of w that ||w'|| < eta ||w||, where the computed
// w' has lost orthogonality to the basis.
__global__ void k_reorth_gate(GmresScalars *S, int j, int m, double eta2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double before = S->H[(int64_t)j * (m + 1) + j + 1].re;
  const int need = S->nrm2.re < eta2 * before;
  S->reorth = need;
  S->reorth_count += need;
}

// ------------------------------------------------------ Bi-CGSTAB pieces
// pair dots: d_q = sum conj(x_q) y_q for q < npairs (<= 2)
template <typename R>
__global__ __launch_bounds__(BS) void k_pairdot(const cplx<R> *__restrict__ x0, const cplx<R> *__restrict__ y0,
                                                const cplx<R> *__restrict__ x1, const cplx<R> *__restrict__ y1,
                                                int npairs, int64_t n, cplx<double> *partials) {
  __shared__ cplx<double> lds[BS / 64];
  cplx<double> a0 = mk<double>(0, 0), a1 = mk<double>(0, 0);
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) {
    a0 = a0 + conjg(cvt<double>(x0[p])) * cvt<double>(y0[p]);
    if (npairs > 1) a1 = a1 + conjg(cvt<double>(x1[p])) * cvt<double>(y1[p]);
  }
  cplx<double> s0 = block_sum(a0, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s0;
  if (npairs > 1) {
    __syncthreads();
    cplx<double> s1 = block_sum(a1, lds);
    if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = s1;
  }
}

// final reduction of pair dots and the Bi-CGSTAB scalar recurrence (one
// block per right-hand side)
template <bool MR>
__global__ __launch_bounds__(BS) void k_bicg_final(const cplx<double> *__restrict__ partials, int nblocks,
                                                   int npairs, BicgScalars *S, int mode, RhsSet rs) {
  __shared__ cplx<double> lds[BS / 64];
  if constexpr (MR) {
    const int64_t q = rhs_index(rs);
    partials += q * kRhsPartials;
    S += q;
  }
  cplx<double> d[2] = {mk<double>(0, 0), mk<double>(0, 0)};
  for (int q = 0; q < npairs; q++) {
    cplx<double> s = strided_sum(partials + (int64_t)q * nblocks, nblocks);
    d[q] = block_sum(s, lds);
    __syncthreads();
  }
  if (threadIdx.x == 0) bicg_update(S, mode, d[0], d[1]);
}

// p = r + beta (p - omega v)
template <typename R, bool MR>
__global__ __launch_bounds__(BS) void k_bicg_p(cplx<R> *__restrict__ p, const cplx<R> *__restrict__ r,
                                               const cplx<R> *__restrict__ v, int64_t n, const BicgScalars *S,
                                               RhsSet rs) {
  if constexpr (MR) {
    const int64_t q = rhs_index(rs), sn = rhs_stride(n);
    p += q * sn;
    r += q * sn;
    v += q * sn;
    S += q;
  }
  const cplx<R> beta = cvt<R>(S->beta), omega = cvt<R>(S->omega);
  for (int64_t q = (int64_t)blockIdx.x * BS + threadIdx.x; q < n; q += (int64_t)gridDim.x * BS)
    p[q] = r[q] + beta * (p[q] - omega * v[q]);
}

// s = r - alpha v
template <typename R, bool MR>
__global__ __launch_bounds__(BS) void k_bicg_s(cplx<R> *__restrict__ s, const cplx<R> *__restrict__ r,
                                               const cplx<R> *__restrict__ v, int64_t n, const BicgScalars *S,
                                               RhsSet rs) {
  if constexpr (MR) {
    const int64_t q = rhs_index(rs), sn = rhs_stride(n);
    s += q * sn;
    r += q * sn;
    v += q * sn;
    S += q;
  }
  const cplx<R> alpha = cvt<R>(S->alpha);
  for (int64_t q = (int64_t)blockIdx.x * BS + threadIdx.x; q < n; q += (int64_t)gridDim.x * BS)
    s[q] = r[q] - alpha * v[q];
}

// x += alpha ph + omega sh ; r = s - omega t ; ||r||^2 and (r^, r) reduced by
// the last block into est and the next step's beta
template <typename R, typename RZ, bool MR>
__global__ __launch_bounds__(BS) void k_bicg_xr(cplx<R> *__restrict__ x, const cplx<RZ> *__restrict__ ph,
                                                const cplx<RZ> *__restrict__ sh, cplx<R> *__restrict__ r,
                                                const cplx<R> *__restrict__ s, const cplx<R> *__restrict__ t,
                                                const cplx<R> *__restrict__ rh, int64_t n, BicgScalars *S,
                                                cplx<double> *partials, RhsSet rs) {
  __shared__ cplx<double> lds[BS / 64];
  if constexpr (MR) {
    const int64_t q = rhs_index(rs), sn = rhs_stride(n);
    x += q * sn;
    ph += q * sn;
    sh += q * sn;
    r += q * sn;
    s += q * sn;
    t += q * sn;
    rh += q * sn;
    S += q;
    partials += q * kRhsPartials;
  }
  const cplx<R> alpha = cvt<R>(S->alpha), omega = cvt<R>(S->omega);
  double nrm = 0;
  cplx<double> rr = mk<double>(0, 0);
  for (int64_t q = (int64_t)blockIdx.x * BS + threadIdx.x; q < n; q += (int64_t)gridDim.x * BS) {
    x[q] = x[q] + alpha * cvt<R>(ph[q]) + omega * cvt<R>(sh[q]);
    const cplx<R> rq = s[q] - omega * t[q];
    r[q] = rq;
    const cplx<double> rd = cvt<double>(rq);
    nrm += abs2(rd);
    rr = rr + conjg(cvt<double>(rh[q])) * rd;
  }
  cplx<double> a0 = block_sum(mk<double>(nrm, 0), lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = a0;
  __syncthreads();
  cplx<double> a1 = block_sum(rr, lds);
  if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = a1;
}

// The nested Bi-CGSTAB's r update without x: r = s - omega t with the same
// dot products, and this step's (alpha, omega) kept in coef[0..1] for the
// deferred x update below (the preconditioned directions p^, s^ of the step
// stay in memory until then).
template <typename R>
__global__ __launch_bounds__(BS) void k_bicg_r(cplx<R> *__restrict__ r, const cplx<R> *__restrict__ s,
                                               const cplx<R> *__restrict__ t, const cplx<R> *__restrict__ rh,
                                               int64_t n, const BicgScalars *S, cplx<double> *partials,
                                               cplx<double> *coef) {
  __shared__ cplx<double> lds[BS / 64];
  const cplx<R> omega = cvt<R>(S->omega);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    coef[0] = S->alpha;
    coef[1] = S->omega;
  }
  double nrm = 0;
  cplx<double> rr = mk<double>(0, 0);
  for (int64_t q = (int64_t)blockIdx.x * BS + threadIdx.x; q < n; q += (int64_t)gridDim.x * BS) {
    const cplx<R> rq = s[q] - omega * t[q];
    r[q] = rq;
    const cplx<double> rd = cvt<double>(rq);
    nrm += abs2(rd);
    rr = rr + conjg(cvt<double>(rh[q])) * rd;
  }
  cplx<double> a0 = block_sum(mk<double>(nrm, 0), lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = a0;
  __syncthreads();
  cplx<double> a1 = block_sum(rr, lds);
  if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = a1;
}

// The deferred x update of `count` steps: x += alpha_i p^_i + omega_i s^_i,
// i = 0 .. count - 1 in order, each step the same expression as the one-step
// update (so x is the same), p^_i and s^_i ld elements apart.  The loads of
// a group of steps are all issued before the first is added.
template <typename R>
__global__ __launch_bounds__(BS) void k_bicg_xdefer(cplx<R> *__restrict__ x, const cplx<R> *__restrict__ ph,
                                                    const cplx<R> *__restrict__ sh, int64_t ld, int count,
                                                    const cplx<double> *__restrict__ coef, int64_t n) {
  constexpr int G = 4;
  for (int64_t q = (int64_t)blockIdx.x * BS + threadIdx.x; q < n; q += (int64_t)gridDim.x * BS) {
    cplx<R> acc = x[q];
    for (int i0 = 0; i0 < count; i0 += G) {
      cplx<R> pv[G], sv[G];
#pragma unroll
      for (int g = 0; g < G; g++) {
        const int i = i0 + g < count ? i0 + g : i0;
        pv[g] = ph[(int64_t)i * ld + q];
        sv[g] = sh[(int64_t)i * ld + q];
      }
#pragma unroll
      for (int g = 0; g < G; g++) {
        if (i0 + g >= count) break;
        const cplx<R> alpha = cvt<R>(coef[2 * (i0 + g)]), omega = cvt<R>(coef[2 * (i0 + g) + 1]);
        acc = acc + alpha * pv[g] + omega * sv[g];
      }
    }
    x[q] = acc;
  }
}

// ----------------------------------------------------------- utilities
template <typename RI, typename RO, bool MR>
__global__ __launch_bounds__(BS) void k_cast(const cplx<RI> *__restrict__ x, cplx<RO> *__restrict__ y, int64_t n,
                                             RhsSet rs) {
  if constexpr (MR) {
    const int64_t q = rhs_index(rs) * rhs_stride(n);
    x += q;
    y += q;
  }
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) y[p] = cvt<RO>(x[p]);
}
__global__ __launch_bounds__(BS) void k_cast_real(const double *__restrict__ x, float *__restrict__ y, int64_t n) {
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) y[p] = (float)x[p];
}
__global__ __launch_bounds__(BS) void k_widen_real(const float *__restrict__ x, double *__restrict__ y, int64_t n) {
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) y[p] = (double)x[p];
}
template <typename R>
__global__ __launch_bounds__(BS) void k_zero(cplx<R> *__restrict__ x, int64_t n) {
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) x[p] = mk<R>(0, 0);
}
// y = W x or W^{-1} x, W = w0(i) w1(j) w2(k) (dual cell widths); boundary -> 0
__global__ __launch_bounds__(BS) void k_scale_w(int n0, int n1, int n2, const cplx<double> *__restrict__ w0,
                                                const cplx<double> *__restrict__ w1,
                                                const cplx<double> *__restrict__ w2,
                                                const cplx<double> *__restrict__ x, cplx<double> *__restrict__ y,
                                                int inverse) {
  const int64_t n = (int64_t)n0 * n1 * n2;
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) {
    int i = (int)(p % n0);
    int j = (int)((p / n0) % n1);
    int k = (int)(p / ((int64_t)n0 * n1));
    bool zin = n2 == 1 || (k >= 1 && k <= n2 - 2);
    if (!(i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && zin)) {
      y[p] = mk<double>(0, 0);
      continue;
    }
    cplx<double> wv = w0[i] * w1[j];
    if (n2 > 1) wv = wv * w2[k];
    y[p] = inverse ? cdiv(x[p], wv) : wv * x[p];
  }
}
// y = x on interior nodes, 0 on the Dirichlet boundary (may run in place)
__global__ __launch_bounds__(BS) void k_mask_boundary(int n0, int n1, int n2, const cplx<double> *x,
                                                      cplx<double> *y) {
  const int64_t n = (int64_t)n0 * n1 * n2;
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) {
    int i = (int)(p % n0);
    int j = (int)((p / n0) % n1);
    int k = (int)(p / ((int64_t)n0 * n1));
    bool zin = n2 == 1 || (k >= 1 && k <= n2 - 2);
    bool in = i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && zin;
    y[p] = in ? x[p] : mk<double>(0, 0);
  }
}
// Coupling of the block system: y_i <- y_i - sum_{j != i} k2c[i nb + j] x_j at
// every node (blocks of nn nodes stacked); with b: y_i <- b_i - (that), the
// residual of the coupled system.  The nb values of x at a node stay in
// registers across the i loop.
template <int NB>
__global__ __launch_bounds__(BS) void k_couple(int64_t nn, const double *__restrict__ k2c,
                                               const cplx<double> *__restrict__ x, cplx<double> *y,
                                               const cplx<double> *__restrict__ b) {
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < nn; p += (int64_t)gridDim.x * BS) {
    cplx<double> xv[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) xv[j] = x[j * nn + p];
#pragma unroll
    for (int i = 0; i < NB; i++) {
      cplx<double> acc = y[i * nn + p];
#pragma unroll
      for (int j = 0; j < NB; j++)
        if (j != i) acc = acc - k2c[(int64_t)(i * NB + j) * nn + p] * xv[j];
      y[i * nn + p] = b ? b[i * nn + p] - acc : acc;
    }
  }
}
__global__ __launch_bounds__(BS) void k_grad_k2(const cplx<double> *__restrict__ lam,
                                                const cplx<double> *__restrict__ u, double *__restrict__ g,
                                                int64_t n) {
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) {
    cplx<double> a = lam[p], b = u[p];
    g[p] = a.re * b.re - a.im * b.im;
  }
}
__global__ __launch_bounds__(BS) void k_max_partial(const double *__restrict__ x, int64_t n, double *partials) {
  __shared__ double lds[BS / 64];
  double m = -INFINITY;
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) m = fmax(m, x[p]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = lds[0];
    for (int q = 1; q < BS / 64; q++) r = fmax(r, lds[q]);
    partials[blockIdx.x] = r;
  }
}
__global__ void k_max_final(const double *partials, int nb, double *out) {
  if (threadIdx.x != 0) return;
  double r = -INFINITY;
  for (int q = 0; q < nb; q++) r = fmax(r, partials[q]);
  *out = r;
}
__global__ __launch_bounds__(BS) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n) {
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) dst[p] = src[p];
}
__global__ void k_copy1(const unsigned char *__restrict__ src, unsigned char *__restrict__ dst, int64_t n) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[p] = src[p];
}

inline int grid_for(int64_t n) {
  int64_t b = (n + BS - 1) / BS;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

int reduction_blocks(int64_t n) { return red_blocks(n); }

template <typename RA, typename RB>
void launch_mdot_partial(const cplx<RA> *V, int64_t ldv, int ncols, const cplx<RB> *w, int64_t n,
                         cplx<double> *partials, hipStream_t s, const int *gate) {
  launch_k((k_mdot<RA, RB>), dim3(red_blocks(n)), dim3(BS), 0, s, V, ldv, ncols, w, n, partials, gate);
}

void launch_reduce_cols(const cplx<double> *partials, int64_t n, int ncols, cplx<double> *out, hipStream_t s,
                        const int *gate) {
  launch_k(k_reduce_cols, dim3(ncols), dim3(BS), 0, s, partials, red_blocks(n), out, gate);
}

void launch_mupdate_partial(const cplx<double> *V, int64_t ldv, int ncols, const cplx<double> *h, cplx<double> *w,
                            int64_t n, cplx<double> *partials, hipStream_t s, const int *gate) {
  launch_k(k_mupdate, dim3(red_blocks(n)), dim3(BS), 0, s, V, ldv, ncols, h, w, n, partials, gate);
}

void launch_mdot2_partial(const cplx<double> *V, int64_t ldv, int ncols, const cplx<double> *x,
                          const cplx<double> *w, int64_t n, cplx<double> *partials, hipStream_t s) {
  launch_k(k_mdot2, dim3(red_blocks(n)), dim3(BS), 0, s, V, ldv, ncols, x, w, n, partials);
}

void launch_mupdate2_partial(const cplx<double> *V, int64_t ldv, int ncols, const cplx<double> *d, cplx<double> *x,
                             cplx<double> *w, int64_t n, cplx<double> *partials, cplx<double> *hcol, hipStream_t s) {
  launch_k(k_mupdate2, dim3(red_blocks(n)), dim3(BS), 0, s, V, ldv, ncols, d, x, w, n, partials, hcol);
}

void launch_reorth_gate(GmresScalars *S, int j, int m, double eta2, hipStream_t s) {
  launch_k(k_reorth_gate, dim3(1), dim3(1), 0, s, S, j, m, eta2);
}

template <typename R>
void launch_nrm2sq(const cplx<R> *x, int64_t n, cplx<double> *partials, cplx<double> *out, hipStream_t s) {
  int nb = red_blocks(n);
  launch_k((k_nrm2sq<R>), dim3(nb), dim3(BS), 0, s, x, n, partials);
  launch_k(k_reduce_cols, dim3(1), dim3(BS), 0, s, partials, nb, out, (const int *)nullptr);
}

template <typename RZ>
void launch_lincomb(const cplx<RZ> *Z, int64_t ldz, int ncols, const cplx<double> *y, cplx<double> *x, int64_t n,
                    hipStream_t s) {
  launch_k((k_lincomb<RZ>), dim3(grid_for(n)), dim3(BS), 0, s, Z, ldz, ncols, y, x, n);
}

void launch_scale_dev(cplx<double> *x, int64_t n, const double *scal, hipStream_t s) {
  launch_k(k_scale_dev, dim3(grid_for(n)), dim3(BS), 0, s, x, n, scal);
}
void launch_gmres_start(GmresScalars *S, int m, hipStream_t s) {
  launch_k(k_gmres_start, dim3(1), dim3(1), 0, s, S, m);
}
void launch_gmres_givens(GmresScalars *S, int j, int m, hipStream_t s) {
  launch_k(k_gmres_givens, dim3(1), dim3(1), 0, s, S, j, m);
}
void launch_gmres_backsolve(GmresScalars *S, int k, int m, hipStream_t s) {
  launch_k(k_gmres_backsolve, dim3(1), dim3(1), 0, s, S, k, m);
}

void launch_add_h2(GmresScalars *S, int j, int m, hipStream_t s, const int *gate) {
  launch_k(k_add_h2, dim3(1), dim3(kMaxRestart + 2), 0, s, S, j, m, gate);
}

template <typename R>
void launch_pairdot(const cplx<R> *x0, const cplx<R> *y0, const cplx<R> *x1, const cplx<R> *y1, int npairs, int64_t n,
                    cplx<double> *partials, BicgScalars *S, int mode, hipStream_t s) {
  int nb = red_blocks(n);
  launch_k((k_pairdot<R>), dim3(nb), dim3(BS), 0, s, x0, y0, x1, y1, npairs, n, partials);
  launch_k(k_bicg_final<false>, dim3(1), dim3(BS), 0, s, partials, nb, npairs, S, mode, one_rhs());
}
template <typename R>
void launch_bicg_p(cplx<R> *p, const cplx<R> *r, const cplx<R> *v, int64_t n, const BicgScalars *S, hipStream_t s,
                   const RhsSet &rs) {
  if (multi_rhs(rs)) launch_k((k_bicg_p<R, true>), dim3(grid_for(n), rs.count), dim3(BS), 0, s, p, r, v, n, S, rs);
  else launch_k((k_bicg_p<R, false>), dim3(grid_for(n)), dim3(BS), 0, s, p, r, v, n, S, rs);
}
template <typename R>
void launch_bicg_s(cplx<R> *sv, const cplx<R> *r, const cplx<R> *v, int64_t n, const BicgScalars *S, hipStream_t s,
                   const RhsSet &rs) {
  if (multi_rhs(rs)) launch_k((k_bicg_s<R, true>), dim3(grid_for(n), rs.count), dim3(BS), 0, s, sv, r, v, n, S, rs);
  else launch_k((k_bicg_s<R, false>), dim3(grid_for(n)), dim3(BS), 0, s, sv, r, v, n, S, rs);
}
template <typename R, typename RZ>
void launch_bicg_xr(cplx<R> *x, const cplx<RZ> *ph, const cplx<RZ> *sh, cplx<R> *r, const cplx<R> *sv,
                    const cplx<R> *t, const cplx<R> *rh, int64_t n, cplx<double> *partials, BicgScalars *S,
                    hipStream_t s, const RhsSet &rs) {
  const int nb = red_blocks(n);
  if (multi_rhs(rs)) {
    launch_k((k_bicg_xr<R, RZ, true>), dim3(nb, rs.count), dim3(BS), 0, s, x, ph, sh, r, sv, t, rh, n, S, partials,
             rs);
    launch_k(k_bicg_final<true>, dim3(1, rs.count), dim3(BS), 0, s, partials, nb, 2, S, (int)kBicgNormRho, rs);
  } else {
    launch_k((k_bicg_xr<R, RZ, false>), dim3(nb), dim3(BS), 0, s, x, ph, sh, r, sv, t, rh, n, S, partials, rs);
    launch_k(k_bicg_final<false>, dim3(1), dim3(BS), 0, s, partials, nb, 2, S, (int)kBicgNormRho, rs);
  }
}

template <typename R>
void launch_bicg_r(cplx<R> *r, const cplx<R> *sv, const cplx<R> *t, const cplx<R> *rh, int64_t n,
                   cplx<double> *partials, BicgScalars *S, cplx<double> *coef, hipStream_t s) {
  const int nb = red_blocks(n);
  launch_k((k_bicg_r<R>), dim3(nb), dim3(BS), 0, s, r, sv, t, rh, n, (const BicgScalars *)S, partials, coef);
  launch_k(k_bicg_final<false>, dim3(1), dim3(BS), 0, s, partials, nb, 2, S, (int)kBicgNormRho, one_rhs());
}
template <typename R>
void launch_bicg_xdefer(cplx<R> *x, const cplx<R> *ph, const cplx<R> *sh, int64_t ld, int count,
                        const cplx<double> *coef, int64_t n, hipStream_t s) {
  launch_k((k_bicg_xdefer<R>), dim3(grid_for(n)), dim3(BS), 0, s, x, ph, sh, ld, count, coef, n);
}
template void launch_bicg_r<float>(cplx<float> *, const cplx<float> *, const cplx<float> *, const cplx<float> *,
                                   int64_t, cplx<double> *, BicgScalars *, cplx<double> *, hipStream_t);
template void launch_bicg_r<double>(cplx<double> *, const cplx<double> *, const cplx<double> *,
                                    const cplx<double> *, int64_t, cplx<double> *, BicgScalars *, cplx<double> *,
                                    hipStream_t);
template void launch_bicg_xdefer<float>(cplx<float> *, const cplx<float> *, const cplx<float> *, int64_t, int,
                                        const cplx<double> *, int64_t, hipStream_t);
template void launch_bicg_xdefer<double>(cplx<double> *, const cplx<double> *, const cplx<double> *, int64_t, int,
                                         const cplx<double> *, int64_t, hipStream_t);

void launch_bicg_final(const cplx<double> *partials, int nblocks, int npairs, BicgScalars *S, int mode,
                       hipStream_t s, const RhsSet &rs) {
  if (multi_rhs(rs))
    launch_k(k_bicg_final<true>, dim3(1, rs.count), dim3(BS), 0, s, partials, nblocks, npairs, S, mode, rs);
  else
    launch_k(k_bicg_final<false>, dim3(1), dim3(BS), 0, s, partials, nblocks, npairs, S, mode, rs);
}

template <typename RI, typename RO>
void launch_cast(const cplx<RI> *x, cplx<RO> *y, int64_t n, hipStream_t s, const RhsSet &rs) {
  if (multi_rhs(rs)) launch_k((k_cast<RI, RO, true>), dim3(grid_for(n), rs.count), dim3(BS), 0, s, x, y, n, rs);
  else launch_k((k_cast<RI, RO, false>), dim3(grid_for(n)), dim3(BS), 0, s, x, y, n, rs);
}
void launch_cast_real(const double *x, float *y, int64_t n, hipStream_t s) {
  launch_k(k_cast_real, dim3(grid_for(n)), dim3(BS), 0, s, x, y, n);
}
void launch_widen_real(const float *x, double *y, int64_t n, hipStream_t s) {
  launch_k(k_widen_real, dim3(grid_for(n)), dim3(BS), 0, s, x, y, n);
}
template <typename R>
void launch_zero(cplx<R> *x, int64_t n, hipStream_t s) {
  launch_k((k_zero<R>), dim3(grid_for(n)), dim3(BS), 0, s, x, n);
}
void launch_scale_w(int n0, int n1, int n2, const cplx<double> *w0, const cplx<double> *w1, const cplx<double> *w2,
                    const cplx<double> *x, cplx<double> *y, bool inverse, hipStream_t s) {
  int64_t n = (int64_t)n0 * n1 * n2;
  launch_k(k_scale_w, dim3(grid_for(n)), dim3(BS), 0, s, n0, n1, n2, w0, w1, w2, x, y, inverse ? 1 : 0);
}
void launch_mask_boundary(int n0, int n1, int n2, const cplx<double> *x, cplx<double> *y, hipStream_t s) {
  int64_t n = (int64_t)n0 * n1 * n2;
  launch_k(k_mask_boundary, dim3(grid_for(n)), dim3(BS), 0, s, n0, n1, n2, x, y);
}
template <int NB>
void launch_couple_nb(int64_t nn, const double *k2c, const cplx<double> *x, cplx<double> *y, const cplx<double> *b,
                      hipStream_t s) {
  launch_k((k_couple<NB>), dim3(grid_for(nn)), dim3(BS), 0, s, nn, k2c, x, y, b);
}
void launch_couple(int nb, int64_t nn, const double *k2c, const cplx<double> *x, cplx<double> *y,
                   const cplx<double> *b, hipStream_t s) {
  switch (nb) {
    case 1: launch_couple_nb<1>(nn, k2c, x, y, b, s); break;
    case 2: launch_couple_nb<2>(nn, k2c, x, y, b, s); break;
    case 3: launch_couple_nb<3>(nn, k2c, x, y, b, s); break;
    case 4: launch_couple_nb<4>(nn, k2c, x, y, b, s); break;
    case 5: launch_couple_nb<5>(nn, k2c, x, y, b, s); break;
    case 6: launch_couple_nb<6>(nn, k2c, x, y, b, s); break;
    case 7: launch_couple_nb<7>(nn, k2c, x, y, b, s); break;
    default: launch_couple_nb<8>(nn, k2c, x, y, b, s); break;
  }
}
void launch_grad_k2(const cplx<double> *lam, const cplx<double> *u, double *g, int64_t n, hipStream_t s) {
  launch_k(k_grad_k2, dim3(grid_for(n)), dim3(BS), 0, s, lam, u, g, n);
}
void launch_max_real(const double *x, int64_t n, double *partials, double *out, hipStream_t s) {
  int nb = red_blocks(n);
  launch_k(k_max_partial, dim3(nb), dim3(BS), 0, s, x, n, partials);
  launch_k(k_max_final, dim3(1), dim3(1), 0, s, partials, nb, out);
}
void launch_empty(hipStream_t s) { launch_k(k_empty, dim3(1), dim3(64), 0, s); }

void launch_copy_bytes(const void *src, void *dst, size_t bytes, hipStream_t s) {
  if (((uintptr_t)src % 16) == 0 && ((uintptr_t)dst % 16) == 0 && bytes % 16 == 0) {
    int64_t n = (int64_t)(bytes / 16);
    int64_t b = (n + BS - 1) / BS;
    if (b > 65536) b = 65536;
    launch_k(k_copy16, dim3((unsigned)b), dim3(BS), 0, s, (const uint4 *)src, (uint4 *)dst, n);
  } else {
    int64_t n = (int64_t)bytes;
    launch_k(k_copy1, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const unsigned char *)src,
                       (unsigned char *)dst, n);
  }
}

template void launch_mdot_partial<double, double>(const cplx<double> *, int64_t, int, const cplx<double> *, int64_t,
                                                  cplx<double> *, hipStream_t, const int *);
template void launch_nrm2sq<double>(const cplx<double> *, int64_t, cplx<double> *, cplx<double> *, hipStream_t);
template void launch_nrm2sq<float>(const cplx<float> *, int64_t, cplx<double> *, cplx<double> *, hipStream_t);
template void launch_lincomb<double>(const cplx<double> *, int64_t, int, const cplx<double> *, cplx<double> *, int64_t,
                                     hipStream_t);
template void launch_lincomb<float>(const cplx<float> *, int64_t, int, const cplx<double> *, cplx<double> *, int64_t,
                                    hipStream_t);
template void launch_pairdot<double>(const cplx<double> *, const cplx<double> *, const cplx<double> *,
                                     const cplx<double> *, int, int64_t, cplx<double> *, BicgScalars *, int,
                                     hipStream_t);
template void launch_pairdot<float>(const cplx<float> *, const cplx<float> *, const cplx<float> *,
                                    const cplx<float> *, int, int64_t, cplx<double> *, BicgScalars *, int, hipStream_t);
template void launch_bicg_p<double>(cplx<double> *, const cplx<double> *, const cplx<double> *, int64_t,
                                    const BicgScalars *, hipStream_t, const RhsSet &);
template void launch_bicg_p<float>(cplx<float> *, const cplx<float> *, const cplx<float> *, int64_t,
                                   const BicgScalars *, hipStream_t, const RhsSet &);
template void launch_bicg_s<double>(cplx<double> *, const cplx<double> *, const cplx<double> *, int64_t,
                                    const BicgScalars *, hipStream_t, const RhsSet &);
template void launch_bicg_s<float>(cplx<float> *, const cplx<float> *, const cplx<float> *, int64_t,
                                   const BicgScalars *, hipStream_t, const RhsSet &);
template void launch_bicg_xr<double, double>(cplx<double> *, const cplx<double> *, const cplx<double> *, cplx<double> *,
                                             const cplx<double> *, const cplx<double> *, const cplx<double> *, int64_t,
                                             cplx<double> *, BicgScalars *, hipStream_t, const RhsSet &);
template void launch_bicg_xr<double, float>(cplx<double> *, const cplx<float> *, const cplx<float> *, cplx<double> *,
                                            const cplx<double> *, const cplx<double> *, const cplx<double> *, int64_t,
                                            cplx<double> *, BicgScalars *, hipStream_t, const RhsSet &);
template void launch_bicg_xr<float, float>(cplx<float> *, const cplx<float> *, const cplx<float> *, cplx<float> *,
                                           const cplx<float> *, const cplx<float> *, const cplx<float> *, int64_t,
                                           cplx<double> *, BicgScalars *, hipStream_t, const RhsSet &);
template void launch_cast<double, float>(const cplx<double> *, cplx<float> *, int64_t, hipStream_t, const RhsSet &);
template void launch_cast<float, double>(const cplx<float> *, cplx<double> *, int64_t, hipStream_t, const RhsSet &);
template void launch_zero<double>(cplx<double> *, int64_t, hipStream_t);
template void launch_zero<float>(cplx<float> *, int64_t, hipStream_t);

}  // namespace ecs
