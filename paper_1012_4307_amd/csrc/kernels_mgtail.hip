// kernels_mgtail.hip -- the coarse end of a general multigrid cycle in one
// workgroup (bin Zubair, Reps, Vanroose, Sec. 4.2, Algorithm 1 with any cycle
// indices gamma_f, gamma_c, omega-Jacobi or red-black relaxation and nu1 / nu2
// sweeps; 2D).
//
// The F cycles of the CSL and CSG set-ups of Sec. 5 (F_1^2 .. F_1^4) visit the
// coarse levels many times per cycle, and on grids of a few hundred nodes a
// launch per sweep, residual/restriction or prolongation costs far more than
// its arithmetic.  The host unrolls the recursion of Algorithm 1 from the
// tail's first level down into a list of level operations (a schedule, see
// ecs_internal.h for the encoding); this kernel keeps every level vector of the
// tail in LDS and runs the schedule, with one workgroup barrier after each
// operation.  Global memory is read once at the start (the first level's
// right-hand side and, for a cycle started from a guess, its iterate; the
// packed weights and inverse diagonals; the coarsest inverse) and written once
// at the end (the first level's result).
#include "ecs_internal.h"

namespace ecs {

namespace {

constexpr int ST = 1024;  // threads of the workgroup

template <typename R>
struct SchedLds {
  cplx<R> pk[kSchedPack];   // per level: xm[n0] xp[n0] ym[n1] yp[n1] dinv[n0 n1]
  cplx<R> b[kTailCap];      // right-hand sides
  cplx<R> u[2][kTailCap];   // iterates; omega-Jacobi alternates between the two
  cplx<R> mi[kTailMinv];    // the coarsest inverse (transposed) when it fits
};

template <typename R>
struct LevelView {
  int n0, n1, no;
  const cplx<R> *xm, *xp, *ym, *yp, *dv;
};

template <typename R>
__device__ __forceinline__ LevelView<R> level_view(const SchedArgs<R> &a, const SchedLds<R> &S, int k) {
  LevelView<R> v;
  v.n0 = a.n0[k];
  v.n1 = a.n1[k];
  v.no = a.noff[k];
  v.xm = S.pk + a.pko[k];
  v.xp = v.xm + v.n0;
  v.ym = v.xp + v.n0;
  v.yp = v.ym + v.n1;
  v.dv = v.yp + v.n1;
  return v;
}

// 1 / z, for the diagonal of M from its stored inverse (residual only)
template <typename R>
__device__ __forceinline__ cplx<R> recip(cplx<R> z) {
  const R s = R(1) / (z.re * z.re + z.im * z.im);
  return mk<R>(z.re * s, -z.im * s);
}

// row of node p of an n0-wide level from a float reciprocal (exact here: the
// levels hold at most kTailCap nodes, so the product stays far from an
// integer boundary)
__device__ __forceinline__ int row_of(int p, float inv) { return (int)(((float)p + 0.5f) * inv); }

// x = M_C^{-1} b on the coarsest level: tpr lanes per row of the inverse,
// partial sums combined across the row's lanes; unknowns are the interior
// nodes in row-major order
template <typename R, typename M>
__device__ __forceinline__ void dense_solve(int nu, int tpr, const M *mi, const cplx<R> *b, cplx<R> *x, int n0) {
  const int tid = threadIdx.x, ni = n0 - 2, rows = ST / tpr;
  // node of unknown c from a float reciprocal (exact: c < 1024)
  const float inv = 1.0f / (float)ni;
  auto node = [&](int c) {
    const int r = (int)(((float)c + 0.5f) * inv);
    return (r + 1) * n0 + (c - r * ni) + 1;
  };
  for (int r0 = 0; r0 < nu; r0 += rows) {
    const int r = r0 + tid / tpr;
    cplx<R> acc = mk<R>(0, 0);
    if (r < nu) {
#pragma unroll 4
      for (int c = tid % tpr; c < nu; c += tpr) acc = acc + mi[(int64_t)c * nu + r] * b[node(c)];
    }
    for (int m = tpr >> 1; m >= 1; m >>= 1) {
      acc.re += __shfl_xor(acc.re, m, 64);
      acc.im += __shfl_xor(acc.im, m, 64);
    }
    if (r < nu && tid % tpr == 0) x[node(r)] = acc;
  }
}

template <typename R>
__global__ __launch_bounds__(ST) void k_sched_tail(SchedArgs<R> a) {
  __shared__ SchedLds<R> S;
  const int tid = threadIdx.x;
  const R om = a.omega, om1 = R(1) - a.omega;
  const bool minv_lds = a.nunk * a.nunk <= kTailMinv;

  // setup: one pass of loads and stores
  {
    const int ntot = a.noff[a.nl], n00 = a.n0[0], nn0 = n00 * a.n1[0];
    const float inv0 = 1.0f / (float)n00;
    for (int x = tid; x < a.pack_len; x += ST) S.pk[x] = a.pack[x];
    if (minv_lds)
      for (int x = tid; x < a.nunk * a.nunk; x += ST) S.mi[x] = a.minvT[x];
    for (int x = tid; x < ntot; x += ST) {
      cplx<R> bv = mk<R>(0, 0), uv = mk<R>(0, 0);
      if (x < nn0) {
        const int j = row_of(x, inv0), i = x - j * n00;
        const bool in = i >= 1 && i <= n00 - 2 && j >= 1 && j <= a.n1[0] - 2;
        if (in) {
          bv = a.b_in[x];
          if (a.u_in) uv = a.u_in[x];
        }
      }
      S.b[x] = bv;
      S.u[0][x] = uv;
      S.u[1][x] = mk<R>(0, 0);
    }
  }
  __syncthreads();

  // the host ends every schedule with kSchedEnd; the bound only guarantees
  // termination
  for (int pc = 0; pc < a.prog_len; pc++) {
    const uint32_t op = a.prog[pc];
    const int code = op & 15, k = (op >> 4) & 15;
    const bool zg = (op >> 8) & 1;
    const int f0 = (op >> 9) & 1, f1 = (op >> 10) & 1;
    if (code == kSchedEnd) {
      const int nn0 = a.n0[0] * a.n1[0];
      for (int x = tid; x < nn0; x += ST) a.u_out[x] = S.u[f0][x];
      break;
    }
    const LevelView<R> L = level_view(a, S, k);
    const int n0 = L.n0, n1 = L.n1, nn = n0 * n1;
    const float inv = 1.0f / (float)n0;
    const cplx<R> *b = S.b + L.no;
    if (code == kSchedJacobi) {
      // out of place: u[f1] = (1 - w) u[f0] + w D^{-1} (b + offd u[f0]);
      // a zero guess reads nothing: u[f1] = w D^{-1} b
      const cplx<R> *us = S.u[f0] + L.no;
      cplx<R> *ud = S.u[f1] + L.no;
      for (int p = tid; p < nn; p += ST) {
        const int j = row_of(p, inv), i = p - j * n0;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
          cplx<R> v;
          if (zg) {
            v = om * (b[p] * L.dv[p]);
          } else {
            const cplx<R> o = L.xm[i] * us[p - 1] + L.xp[i] * us[p + 1] + L.ym[j] * us[p - n0] + L.yp[j] * us[p + n0];
            v = om1 * us[p] + om * ((b[p] + o) * L.dv[p]);
          }
          ud[p] = v;
        }
      }
    } else if (code == kSchedRB) {
      // one colour (f1: 0 red = (i + j) even, 1 black) in place on u[f0];
      // threads enumerate node pairs (columns 2h, 2h + 1 of a row), one node
      // of each colour.  A zero-guess red pass also writes the black nodes' 0.
      cplx<R> *u = S.u[f0] + L.no;
      const int H = (n0 + 1) >> 1, np = n1 * H;
      const float invH = 1.0f / (float)H;
      for (int q = tid; q < np; q += ST) {
        const int j = row_of(q, invH), h2 = 2 * (q - j * H);
        const int i = h2 + ((j + f1) & 1), p = j * n0 + i;
        const bool in = i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2;
        if (zg) {
          const int io = h2 + ((j + f1 + 1) & 1);
          if (i < n0) u[p] = in ? om * (b[p] * L.dv[p]) : mk<R>(0, 0);
          if (io < n0) u[j * n0 + io] = mk<R>(0, 0);
        } else if (in) {
          const cplx<R> o = L.xm[i] * u[p - 1] + L.xp[i] * u[p + 1] + L.ym[j] * u[p - n0] + L.yp[j] * u[p + n0];
          u[p] = om1 * u[p] + om * ((b[p] + o) * L.dv[p]);
        }
      }
    } else if (code == kSchedResid) {
      // residual of u[f0] into the level's other buffer, then full weighting
      // onto the next level's right-hand side
      const cplx<R> *u = S.u[f0] + L.no;
      cplx<R> *r = S.u[f0 ^ 1] + L.no;
      for (int p = tid; p < nn; p += ST) {
        const int j = row_of(p, inv), i = p - j * n0;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
          const cplx<R> o = L.xm[i] * u[p - 1] + L.xp[i] * u[p + 1] + L.ym[j] * u[p - n0] + L.yp[j] * u[p + n0];
          r[p] = (b[p] + o) - recip(L.dv[p]) * u[p];
        }
      }
      __syncthreads();
      const int c0 = a.n0[k + 1], c1 = a.n1[k + 1], nc = c0 * c1;
      const float invc = 1.0f / (float)c0;
      cplx<R> *bc = S.b + a.noff[k + 1];
      for (int q = tid; q < nc; q += ST) {
        const int J = row_of(q, invc), I = q - J * c0;
        cplx<R> acc = mk<R>(0, 0);
        if (I >= 1 && I <= c0 - 2 && J >= 1 && J <= c1 - 2) {
          const cplx<R> *r0 = r + (2 * J) * n0 + 2 * I;
          acc = R(0.25) * r0[0] + R(0.125) * (r0[-1] + r0[1] + r0[-n0] + r0[n0]) +
                R(0.0625) * (r0[-n0 - 1] + r0[-n0 + 1] + r0[n0 - 1] + r0[n0 + 1]);
        }
        bc[q] = acc;
      }
    } else if (code == kSchedCoarse) {
      cplx<R> *x = S.u[f0] + L.no;
      if (minv_lds) dense_solve(a.nunk, a.tpr, S.mi, b, x, n0);
      else dense_solve(a.nunk, a.tpr, a.minvT, b, x, n0);
    } else if (code == kSchedProlong) {
      // u[f0] += P e, e = u[f1] of the next level (bilinear in index space)
      cplx<R> *u = S.u[f0] + L.no;
      const int c0 = a.n0[k + 1];
      const cplx<R> *e = S.u[f1] + a.noff[k + 1];
      for (int p = tid; p < nn; p += ST) {
        const int j = row_of(p, inv), i = p - j * n0;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
          const cplx<R> *e0 = e + (j >> 1) * c0 + (i >> 1);
          cplx<R> v;
          if ((i & 1) == 0 && (j & 1) == 0) v = e0[0];
          else if ((j & 1) == 0) v = R(0.5) * (e0[0] + e0[1]);
          else if ((i & 1) == 0) v = R(0.5) * (e0[0] + e0[c0]);
          else v = R(0.25) * (e0[0] + e0[1] + e0[c0] + e0[c0 + 1]);
          u[p] = u[p] + v;
        }
      }
    } else if (code == kSchedZero) {
      cplx<R> *u = S.u[f0] + L.no;
      for (int p = tid; p < nn; p += ST) u[p] = mk<R>(0, 0);
    }
    __syncthreads();
  }
}

}  // namespace

template <typename R>
void launch_sched_tail(const SchedArgs<R> &a, hipStream_t s) {
  launch_k((k_sched_tail<R>), dim3(1), dim3(ST), 0, s, a);
}

template void launch_sched_tail<double>(const SchedArgs<double> &, hipStream_t);
template void launch_sched_tail<float>(const SchedArgs<float> &, hipStream_t);

}  // namespace ecs
