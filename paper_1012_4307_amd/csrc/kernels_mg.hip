// kernels_mg.hip -- multigrid components of the ECS Helmholtz preconditioner
// (bin Zubair, Reps, Vanroose, Sec. 3.2 operator, Sec. 4.2 components):
// stencil apply, residual, omega-Jacobi and red-black SOR sweeps, full-weighting
// restriction (fused with the residual), bilinear/trilinear prolongation with
// correction, dense coarsest solve, k^2 injection.
//
// Layout: node-major, x fastest, interleaved complex.  Every kernel maps one
// thread to one node of a (64 x 4) tile of an x-y plane; the z plane (3D) is
// blockIdx.z.  Loads along x are unit stride, so a wave reads 64 consecutive
// nodes (1 KB in FP64) per access.  Boundary nodes carry zeros.
#include "ecs_reduce.h"

namespace ecs {

namespace {

constexpr int TX = 64;
constexpr int TY = 4;

template <typename R>
struct Node {
  int i, j, k;
  int64_t p;
  bool in;        // inside the array
  bool interior;  // not a Dirichlet node
};

// blocks are launched 1D over the (x tiles) x (y tiles) x (z planes) tiles
// of the grid in XCD-aware order; padding blocks get in = false
template <typename R>
__device__ __forceinline__ Node<R> node_of(const Grid<R> &g) {
  Node<R> q;
  const int tx = (g.n0 + TX - 1) / TX, ty = (g.n1 + TY - 1) / TY;
  const int tile = xcd_tile(tx * ty * g.n2);
  const int tt = tile < 0 ? 0 : tile;
  q.i = (tt % tx) * TX + threadIdx.x;
  q.j = ((tt / tx) % ty) * TY + threadIdx.y;
  q.k = tt / (tx * ty);
  q.in = tile >= 0 && q.i < g.n0 && q.j < g.n1;
  q.p = ((int64_t)q.k * g.n1 + q.j) * g.n0 + q.i;
  bool zin = g.n2 == 1 || (q.k >= 1 && q.k <= g.n2 - 2);
  q.interior = q.in && q.i >= 1 && q.i <= g.n0 - 2 && q.j >= 1 && q.j <= g.n1 - 2 && zin;
  return q;
}

// diagonal of M at an interior node
template <typename R>
__device__ __forceinline__ cplx<R> diag_at(const Grid<R> &g, int i, int j, int k, int64_t p) {
  cplx<R> d = g.cm0[i] + g.cp0[i] + g.cm1[j] + g.cp1[j];
  if (g.n2 > 1) d = d + g.cm2[k] + g.cp2[k];
  return d + (g.k2[p] * g.beta + g.c);
}

// off-diagonal part: sum of (cm u_{p-s} + cp u_{p+s}) so that M u = D u - offd
template <typename R, typename RI>
__device__ __forceinline__ cplx<R> offd_at(const Grid<R> &g, const cplx<RI> *__restrict__ u, int i, int j, int k,
                                           int64_t p) {
  const int64_t s1 = g.n0;
  cplx<R> o = g.cm0[i] * cvt<R>(u[p - 1]) + g.cp0[i] * cvt<R>(u[p + 1]);
  o = o + g.cm1[j] * cvt<R>(u[p - s1]) + g.cp1[j] * cvt<R>(u[p + s1]);
  if (g.n2 > 1) {
    const int64_t s2 = (int64_t)g.n0 * g.n1;
    o = o + g.cm2[k] * cvt<R>(u[p - s2]) + g.cp2[k] * cvt<R>(u[p + s2]);
  }
  return o;
}

// The same two quantities with the dimension fixed at compile time (no
// branches between the loads, so a thread's loads are all in flight together).
template <typename R, int DIM>
__device__ __forceinline__ cplx<R> diag_d(const Grid<R> &g, int i, int j, int k, int64_t p) {
  cplx<R> d = g.cm0[i] + g.cp0[i] + g.cm1[j] + g.cp1[j];
  if constexpr (DIM == 3) d = d + g.cm2[k] + g.cp2[k];
  return d + (g.k2[p] * g.beta + g.c);
}
template <typename R, int DIM>
__device__ __forceinline__ cplx<R> offd_d(const Grid<R> &g, const cplx<R> *__restrict__ u, int i, int j, int k,
                                          int64_t p) {
  const int64_t s1 = g.n0;
  cplx<R> o = g.cm0[i] * u[p - 1] + g.cp0[i] * u[p + 1] + g.cm1[j] * u[p - s1] + g.cp1[j] * u[p + s1];
  if constexpr (DIM == 3) {
    const int64_t s2 = (int64_t)g.n0 * g.n1;
    o = o + g.cm2[k] * u[p - s2] + g.cp2[k] * u[p + s2];
  }
  return o;
}

template <typename R>
dim3 grid_of(const Grid<R> &g) {
  return dim3(xcd_padded(((g.n0 + TX - 1) / TX) * ((g.n1 + TY - 1) / TY) * g.n2));
}

// y = M x; the input may be stored in a lower precision than the arithmetic
// (an FP32 preconditioned vector fed to the FP64 operator)
template <typename R, typename RI, typename RO>
__global__ __launch_bounds__(256) void k_apply(Grid<R> g, const cplx<RI> *__restrict__ x, cplx<RO> *__restrict__ y) {
  Node<R> q = node_of(g);
  if (!q.in) return;
  if (!q.interior) {
    y[q.p] = mk<RO>(0, 0);
    return;
  }
  cplx<R> v = diag_at(g, q.i, q.j, q.k, q.p) * cvt<R>(x[q.p]) - offd_at<R, RI>(g, x, q.i, q.j, q.k, q.p);
  y[q.p] = cvt<RO>(v);
}

template <typename R>
__global__ __launch_bounds__(256) void k_residual(Grid<R> g, const cplx<R> *__restrict__ b,
                                                  const cplx<R> *__restrict__ u, cplx<R> *__restrict__ r) {
  Node<R> q = node_of(g);
  if (!q.in) return;
  if (!q.interior) {
    r[q.p] = mk<R>(0, 0);
    return;
  }
  r[q.p] = b[q.p] - (diag_at(g, q.i, q.j, q.k, q.p) * u[q.p] - offd_at<R, R>(g, u, q.i, q.j, q.k, q.p));
}

// omega-Jacobi, out of place: out = u + omega D^{-1} (b - M u); zero_guess
// skips reading u (u == 0): out = omega D^{-1} b
template <typename R>
__global__ __launch_bounds__(256) void k_jacobi(Grid<R> g, const cplx<R> *__restrict__ b,
                                                const cplx<R> *__restrict__ u, cplx<R> *__restrict__ out, R omega,
                                                int zero_guess) {
  Node<R> q = node_of(g);
  if (!q.in) return;
  if (!q.interior) {
    out[q.p] = mk<R>(0, 0);
    return;
  }
  // uniform branches first, then every load of the path, then the arithmetic
  if (zero_guess) {
    const cplx<R> bv = b[q.p];
    const cplx<R> d = g.n2 > 1 ? diag_d<R, 3>(g, q.i, q.j, q.k, q.p) : diag_d<R, 2>(g, q.i, q.j, q.k, q.p);
    out[q.p] = omega * cdiv(bv, d);
  } else {
    const cplx<R> bv = b[q.p], u0 = u[q.p];
    cplx<R> d, o;
    if (g.n2 > 1) {
      d = diag_d<R, 3>(g, q.i, q.j, q.k, q.p);
      o = offd_d<R, 3>(g, u, q.i, q.j, q.k, q.p);
    } else {
      d = diag_d<R, 2>(g, q.i, q.j, q.k, q.p);
      o = offd_d<R, 2>(g, u, q.i, q.j, q.k, q.p);
    }
    out[q.p] = u0 + omega * cdiv(bv - (d * u0 - o), d);
  }
}

// one colour of a red-black SOR sweep, in place: nodes of colour `colour`
// ((i+j+k) & 1) are relaxed; they only couple to the other colour.  With
// zero_guess (u == 0 on entry, red pass) the red nodes get omega D^{-1} b and
// every other node of the array is written as 0, so u needs no clearing.
template <typename R>
__global__ __launch_bounds__(256) void k_rb_colour(Grid<R> g, const cplx<R> *__restrict__ b, cplx<R> *u, R omega,
                                                   int colour, int zero_guess) {
  Node<R> q = node_of(g);
  if (!q.in) return;
  bool mine = q.interior && (((q.i + q.j + q.k) & 1) == colour);
  if (zero_guess) {
    u[q.p] = mine ? omega * cdiv(b[q.p], diag_at(g, q.i, q.j, q.k, q.p)) : mk<R>(0, 0);
    return;
  }
  if (!mine) return;
  const cplx<R> bv = b[q.p], u0 = u[q.p];
  cplx<R> d, o;
  if (g.n2 > 1) {
    d = diag_d<R, 3>(g, q.i, q.j, q.k, q.p);
    o = offd_d<R, 3>(g, u, q.i, q.j, q.k, q.p);
  } else {
    d = diag_d<R, 2>(g, q.i, q.j, q.k, q.p);
    o = offd_d<R, 2>(g, u, q.i, q.j, q.k, q.p);
  }
  u[q.p] = u0 + omega * cdiv(bv - (d * u0 - o), d);
}

// full weighting of a fine-grid vector onto the coarse interior, index space
// tensor product of [1 2 1]/4 per active axis
template <typename R>
__global__ __launch_bounds__(256) void k_restrict(Grid<R> f, Grid<R> c, const cplx<R> *__restrict__ rf,
                                                  cplx<R> *__restrict__ rc) {
  Node<R> q = node_of(c);
  if (!q.in) return;
  if (!q.interior) {
    rc[q.p] = mk<R>(0, 0);
    return;
  }
  const int64_t s1 = f.n0, s2 = (int64_t)f.n0 * f.n1;
  const int fk = f.n2 > 1 ? 2 * q.k : 0;
  const int64_t pf = ((int64_t)fk * f.n1 + 2 * q.j) * f.n0 + 2 * q.i;
  const R wgt[3] = {R(0.25), R(0.5), R(0.25)};
  cplx<R> acc = mk<R>(0, 0);
  const int kz = f.n2 > 1 ? 1 : 0;
  for (int dz = -kz; dz <= kz; dz++) {
    R wz = kz ? wgt[dz + 1] : R(1);
    for (int dy = -1; dy <= 1; dy++)
      for (int dx = -1; dx <= 1; dx++) {
        R w = wz * wgt[dy + 1] * wgt[dx + 1];
        acc = acc + w * rf[pf + dz * s2 + dy * s1 + dx];
      }
  }
  rc[q.p] = acc;
}

// fused residual + full weighting: the 3^d fine residuals under the coarse
// node are recomputed from u (no fine residual vector is stored).  Under an
// interior coarse node every one of them is a fine interior node, so the
// loops need no tests: fixed trip counts, all loads in flight together.
template <typename R, int DIM>
__device__ __forceinline__ cplx<R> fw_residual(const Grid<R> &f, const cplx<R> *__restrict__ b,
                                               const cplx<R> *__restrict__ u, int I, int J, int K) {
  const R wgt[3] = {R(0.25), R(0.5), R(0.25)};
  cplx<R> acc = mk<R>(0, 0);
#pragma unroll
  for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); dz++) {
    const int fk = DIM == 3 ? 2 * K + dz : 0;
    const R wz = DIM == 3 ? wgt[dz + 1] : R(1);
#pragma unroll
    for (int dy = -1; dy <= 1; dy++) {
      const int fj = 2 * J + dy;
#pragma unroll
      for (int dx = -1; dx <= 1; dx++) {
        const int fi = 2 * I + dx;
        const int64_t p = ((int64_t)fk * f.n1 + fj) * f.n0 + fi;
        const cplx<R> r = b[p] - (diag_d<R, DIM>(f, fi, fj, fk, p) * u[p] - offd_d<R, DIM>(f, u, fi, fj, fk, p));
        acc = acc + (wz * wgt[dy + 1] * wgt[dx + 1]) * r;
      }
    }
  }
  return acc;
}

template <typename R>
__global__ __launch_bounds__(256) void k_residual_restrict(Grid<R> f, Grid<R> c, const cplx<R> *__restrict__ b,
                                                           const cplx<R> *__restrict__ u, cplx<R> *__restrict__ rc) {
  Node<R> q = node_of(c);
  if (!q.in) return;
  if (!q.interior) {
    rc[q.p] = mk<R>(0, 0);
    return;
  }
  rc[q.p] = f.n2 > 1 ? fw_residual<R, 3>(f, b, u, q.i, q.j, q.k) : fw_residual<R, 2>(f, b, u, q.i, q.j, q.k);
}

// u_out = u_in + P ec on the fine interior (bilinear / trilinear in index
// space); in place when u_out == u_in, else the boundary of u_out gets 0
template <typename R>
__global__ __launch_bounds__(256) void k_prolong_add(Grid<R> f, Grid<R> c, const cplx<R> *__restrict__ ec,
                                                     const cplx<R> *u_in, cplx<R> *u_out) {
  Node<R> q = node_of(f);
  if (!q.in) return;
  if (!q.interior) {
    if (u_out != u_in) u_out[q.p] = mk<R>(0, 0);
    return;
  }
  int ci[3][2], nc[3];
  R cw[3][2];
  const int fi[3] = {q.i, q.j, q.k};
  const int dims = f.n2 > 1 ? 3 : 2;
  for (int a = 0; a < 3; a++) {
    if (a >= dims) {
      nc[a] = 1; ci[a][0] = 0; cw[a][0] = R(1);
    } else if ((fi[a] & 1) == 0) {
      nc[a] = 1; ci[a][0] = fi[a] >> 1; cw[a][0] = R(1);
    } else {
      nc[a] = 2; ci[a][0] = fi[a] >> 1; ci[a][1] = (fi[a] >> 1) + 1; cw[a][0] = cw[a][1] = R(0.5);
    }
  }
  cplx<R> e = mk<R>(0, 0);
  for (int cz = 0; cz < nc[2]; cz++)
    for (int cy = 0; cy < nc[1]; cy++)
      for (int cx = 0; cx < nc[0]; cx++) {
        int64_t pc = ((int64_t)ci[2][cz] * c.n1 + ci[1][cy]) * c.n0 + ci[0][cx];
        e = e + (cw[0][cx] * cw[1][cy] * cw[2][cz]) * ec[pc];
      }
  u_out[q.p] = u_in[q.p] + e;
}

// (P ec) at fine node (i, j) of a 2D level: bilinear in index space; zero on
// the fine boundary because ec is zero on the coarse boundary.  Branch-free:
// the mean of the four coarse nodes (I0 or I0 + 1) x (J0 or J0 + 1), where an
// even index takes the same coarse node twice (never outside the level).
template <typename R>
__device__ __forceinline__ cplx<R> prolong_at(const cplx<R> *__restrict__ ec, int c0, int i, int j) {
  const int I0 = i >> 1, J0 = j >> 1, I1 = I0 + (i & 1), J1 = J0 + (j & 1);
  const cplx<R> *r0 = ec + (int64_t)J0 * c0, *r1 = ec + (int64_t)J1 * c0;
  return R(0.25) * ((r0[I0] + r0[I1]) + (r1[I0] + r1[I1]));
}

// 2D coarse-grid correction fused with the first omega-Jacobi post-sweep, out
// of place: out = J(u + P ec).  The corrected iterate at the node's four
// neighbours is formed on the fly (u and ec are zero on their boundaries).
template <typename R>
__global__ __launch_bounds__(256) void k_prolong_jacobi(Grid<R> f, Grid<R> c, const cplx<R> *__restrict__ ec,
                                                        const cplx<R> *__restrict__ b,
                                                        const cplx<R> *__restrict__ u, cplx<R> *__restrict__ out,
                                                        R omega) {
  Node<R> q = node_of(f);
  if (!q.in) return;
  if (!q.interior) {
    out[q.p] = mk<R>(0, 0);
    return;
  }
  const int i = q.i, j = q.j, n0 = f.n0, c0 = c.n0;
  const int64_t p = q.p;
  const cplx<R> v = u[p] + prolong_at(ec, c0, i, j);
  const cplx<R> vw = u[p - 1] + prolong_at(ec, c0, i - 1, j), ve = u[p + 1] + prolong_at(ec, c0, i + 1, j);
  const cplx<R> vs = u[p - n0] + prolong_at(ec, c0, i, j - 1), vn = u[p + n0] + prolong_at(ec, c0, i, j + 1);
  const cplx<R> o = f.cm0[i] * vw + f.cp0[i] * ve + f.cm1[j] * vs + f.cp1[j] * vn;
  const cplx<R> d = diag_at(f, i, j, 0, p);
  const cplx<R> res = b[p] - (d * v - o);
  out[p] = v + omega * cdiv(res, d);
}

// x = M_C^{-1} b on the coarsest level from the precomputed dense inverse,
// stored transposed (minvT[c * nunk + r] = Minv[r][c]) so that the threads of
// a wave read consecutive entries; b's unknowns are first staged in LDS.
// Thread t writes the t-th unknown and, if node t is a boundary node, its zero.
// One block of 1024 threads (nunk <= 2048 unknowns).
template <typename R, bool MR>
__global__ __launch_bounds__(1024) void k_coarse_solve(int nunk, const cplx<R> *__restrict__ minvT,
                                                       const int *__restrict__ unk, int n0, int n1, int n2,
                                                       const cplx<R> *__restrict__ b, cplx<R> *__restrict__ x,
                                                       RhsSet rs) {
  __shared__ cplx<R> sb[2048];
  const int nn = n0 * n1 * n2;
  if constexpr (MR) {
    const int64_t q = rhs_index(rs) * rhs_stride(nn);  // one block per right-hand side
    b += q;
    x += q;
  }
  for (int t = threadIdx.x; t < nunk; t += blockDim.x) sb[t] = b[unk[t]];
  for (int t = threadIdx.x; t < nn; t += blockDim.x) {
    const int i = t % n0, j = (t / n0) % n1, k = t / (n0 * n1);
    const bool zin = n2 == 1 || (k >= 1 && k <= n2 - 2);
    const bool interior = i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && zin;
    if (!interior) x[t] = mk<R>(0, 0);
  }
  __syncthreads();
  for (int r = threadIdx.x; r < nunk; r += blockDim.x) {
    cplx<R> acc = mk<R>(0, 0);
#pragma unroll 8
    for (int c = 0; c < nunk; c++) acc = acc + minvT[(int64_t)c * nunk + r] * sb[c];
    x[unk[r]] = acc;
  }
}

// y = M x with a fused dot product for Bi-CGSTAB (grid-stride over 64 x 4
// tiles; one thread per node):
//   kBicgAlpha: sum conj(d0) y  -> alpha = rho / (r^, v)
//   kBicgOmega: sum conj(y) d0, sum |y|^2 -> omega = (t, s) / (t, t)
// Per-block partials; a second fixed-order stage (launch_bicg_final) reduces
// them and updates the scalars.
template <typename R, typename RI>
__global__ __launch_bounds__(256) void k_apply_dot(Grid<R> g, const cplx<RI> *__restrict__ x,
                                                   cplx<R> *__restrict__ y, const cplx<R> *__restrict__ d0,
                                                   int mode, cplx<double> *partials, BicgScalars *S) {
  __shared__ cplx<double> lds[4];
  const int tx = (g.n0 + TX - 1) / TX, ty = (g.n1 + TY - 1) / TY;
  const int ntiles = tx * ty * g.n2;
  const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
  cplx<double> a0 = mk<double>(0, 0);
  double a1 = 0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int i = (t % tx) * TX + lx, j = ((t / tx) % ty) * TY + ly, k = t / (tx * ty);
    if (i >= g.n0 || j >= g.n1) continue;
    const int64_t p = ((int64_t)k * g.n1 + j) * g.n0 + i;
    const bool zin = g.n2 == 1 || (k >= 1 && k <= g.n2 - 2);
    cplx<R> v = mk<R>(0, 0);
    if (i >= 1 && i <= g.n0 - 2 && j >= 1 && j <= g.n1 - 2 && zin)
      v = diag_at(g, i, j, k, p) * cvt<R>(x[p]) - offd_at<R, RI>(g, x, i, j, k, p);
    y[p] = v;
    const cplx<double> vd = cvt<double>(v), dd = cvt<double>(d0[p]);
    if (mode == kBicgAlpha) {
      a0 = a0 + conjg(dd) * vd;
    } else {
      a0 = a0 + conjg(vd) * dd;
      a1 += abs2(vd);
    }
  }
  cplx<double> s0 = block_sum(a0, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s0;
  if (mode != kBicgAlpha) {
    __syncthreads();
    cplx<double> s1 = block_sum(mk<double>(a1, 0), lds);
    if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = s1;
  }
}

// 2D y = M x by column strips (the form every 2D matvec of the solve takes):
// a wave owns SX = 62 columns (lanes 1..62; lanes 0 and 63 load the halo
// columns) and SY consecutive rows, with all SY + 2 rows of x it needs in
// registers, the x-neighbours taken from the adjacent lanes.  x is read once
// (plus 2 halo rows per SY), so the pass streams at close to copy speed.  The
// operator's arithmetic is that of k_apply term for term.  MODE fuses the
// Bi-CGSTAB dot products of k_apply_dot (kBicgAlpha / kBicgOmega), 0 = none.
constexpr int SX = 62;

template <typename R, typename RI, typename RO, int MODE, int SY, bool MR = false>
__global__ __launch_bounds__(256) void k_apply2d(Grid<R> g, const cplx<RI> *__restrict__ x, cplx<RO> *__restrict__ y,
                                                 const cplx<R> *__restrict__ d0, cplx<double> *partials, int tiles_x,
                                                 int tiles, RhsSet rs) {
  __shared__ cplx<double> lds[4];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n0 = g.n0, n1 = g.n1;
  if constexpr (MR) {
    const int64_t q = rhs_index(rs), sn = rhs_stride((int64_t)n0 * n1);
    x += q * sn;
    y += q * sn;
    if (MODE != 0) {
      d0 += q * sn;
      partials += q * kRhsPartials;
    }
  }
  const int padded = gridDim.x, b = blockIdx.x;
  const int local = (b % kXcds) * (padded / kXcds) + b / kXcds;  // XCD-aware order within a pass
  cplx<double> a0 = mk<double>(0, 0);
  double a1 = 0;
  for (int t0 = 0; t0 < tiles; t0 += padded) {
    const int tile = t0 + local;
    if (tile >= tiles) continue;
    const int i = (tile % tiles_x) * SX + lane;
    const int j0 = ((tile / tiles_x) * 4 + wv) * SY;
    const bool xin = i < n0;
    const bool xint = i >= 1 && i <= n0 - 2;
    const bool own = xin && ((lane >= 1 && lane <= SX) || i == 0);
    const cplx<R> cxm = xint ? g.cm0[i] : mk<R>(0, 0);
    const cplx<R> cxp = xint ? g.cp0[i] : mk<R>(0, 0);
    // the strip's rows through buffer resources (rows outside the grid and
    // lanes beyond it read 0); the lane's column offsets are fixed
    const int jx = max(j0 - 1, 0), je = min(j0 + SY, n1);
    const __amdgpu_buffer_rsrc_t rx = rows_rsrc(x, jx, min(j0 + SY + 1, n1), n0);
    const __amdgpu_buffer_rsrc_t rk = rows_rsrc(g.k2, j0, je, n0), rd = rows_rsrc(d0, j0, je, n0);
    const __amdgpu_buffer_rsrc_t ry = rows_rsrc(y, j0, je, n0);
    const uint32_t ox = col_off<cplx<RI>>(xin, i), ok = col_off<R>(xin, i), od = col_off<cplx<R>>(xin, i);
    const uint32_t oy = col_off<cplx<RO>>(own, i);
    cplx<R> xv[SY + 2];
#pragma unroll
    for (int r = 0; r < SY + 2; r++)
      xv[r] = cvt<R>(ld_c(rx, ox + row_off<cplx<RI>>(j0 - 1 + r - jx, n0), cplx<RI>()));
    R kv[SY];
    cplx<R> dv[SY];
#pragma unroll
    for (int r = 0; r < SY; r++) {
      kv[r] = ld_r(rk, ok + row_off<R>(r, n0), R());
      dv[r] = MODE != 0 ? ld_c(rd, od + row_off<cplx<R>>(r, n0), cplx<R>()) : mk<R>(0, 0);
    }
#pragma unroll
    for (int r = 0; r < SY; r++) {
      const int jj = j0 + r;
      cplx<R> xl, xr;
      xl.re = __shfl_up(xv[r + 1].re, 1, 64);
      xl.im = __shfl_up(xv[r + 1].im, 1, 64);
      xr.re = __shfl_down(xv[r + 1].re, 1, 64);
      xr.im = __shfl_down(xv[r + 1].im, 1, 64);
      if (jj >= n1) continue;
      const bool yint = jj >= 1 && jj <= n1 - 2;
      const int jc = yint ? jj : 1;
      const cplx<R> cym = yint ? g.cm1[jc] : mk<R>(0, 0), cyp = yint ? g.cp1[jc] : mk<R>(0, 0);
      const cplx<R> d = cxm + cxp + cym + cyp + (kv[r] * g.beta + g.c);
      cplx<R> o = cxm * xl + cxp * xr;
      o = o + cym * xv[r] + cyp * xv[r + 2];
      const cplx<R> v = (xint && yint) ? d * xv[r + 1] - o : mk<R>(0, 0);
      st_c(ry, oy + row_off<cplx<RO>>(r, n0), cvt<RO>(v));
      if (MODE != 0 && own) {
        const cplx<double> vd = cvt<double>(v), dd = cvt<double>(dv[r]);
        if (MODE == kBicgAlpha) {
          a0 = a0 + conjg(dd) * vd;
        } else {
          a0 = a0 + conjg(vd) * dd;
          a1 += abs2(vd);
        }
      }
    }
  }
  if (MODE != 0) {
    cplx<double> s0 = block_sum(a0, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s0;
    if (MODE != kBicgAlpha) {
      __syncthreads();
      cplx<double> s1 = block_sum(mk<double>(a1, 0), lds);
      if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = s1;
    }
  }
}

// strip rows per wave: the x window lives in registers; the dot-product
// variants hold a second operand per row, so they take shorter strips
template <typename R, int MODE>
constexpr int strip_rows() {
  return MODE != 0 ? 8 : (sizeof(R) == 4 ? 16 : 8);
}

template <typename R>
__global__ void k_inject_k2(int n0, int n1, int n2, const double *__restrict__ kf, int f0, int f1, int stride,
                            R *__restrict__ kc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  int k = blockIdx.z;
  if (i >= n0) return;
  int64_t pf = ((int64_t)(n2 > 1 ? k * stride : 0) * f1 + (int64_t)j * stride) * f0 + (int64_t)i * stride;
  kc[((int64_t)k * n1 + j) * n0 + i] = R(kf[pf]);
}

}  // namespace

// 2D launches of the strip kernel: one block (4 waves, 62 x 4 SY nodes) per
// tile while the tile count fits the reduction buffer, grid-stride beyond
// blocks: one per strip tile while the partials (two per block) fit the
// reduction buffer, or a right-hand side's share of it in a batched launch
template <typename R>
void strip_grid(const Grid<R> &g, int sy, int *tiles_x, int *tiles, int *blocks, bool batched = false) {
  *tiles_x = (g.n0 - 1 + SX - 1) / SX;
  *tiles = *tiles_x * ((g.n1 + 4 * sy - 1) / (4 * sy));
  const int cap = batched ? kRhsPartials / 2 : kRedBlocks * (kMaxRestart + 2) / 2;
  *blocks = xcd_padded(*tiles < cap ? *tiles : cap);
}

template <typename R, typename RI, typename RO>
void launch_apply(const Grid<R> &g, const cplx<RI> *x, cplx<RO> *y, hipStream_t s) {
  if (g.n2 == 1) {
    constexpr int sy = strip_rows<R, 0>();
    int tx, tiles, nb;
    strip_grid(g, sy, &tx, &tiles, &nb);
    launch_k((k_apply2d<R, RI, RO, 0, sy>), dim3(nb), dim3(256), 0, s, g, x, y,
                       (const cplx<R> *)nullptr, (cplx<double> *)nullptr, tx, tiles, one_rhs());
    return;
  }
  launch_k((k_apply<R, RI, RO>), grid_of(g), dim3(TX, TY), 0, s, g, x, y);
}
template <typename R>
void launch_residual(const Grid<R> &g, const cplx<R> *b, const cplx<R> *u, cplx<R> *r, hipStream_t s) {
  launch_k((k_residual<R>), grid_of(g), dim3(TX, TY), 0, s, g, b, u, r);
}
template <typename R>
void launch_jacobi(const Grid<R> &g, const cplx<R> *b, const cplx<R> *u, cplx<R> *out, R omega, bool zero_guess,
                   hipStream_t s) {
  launch_k((k_jacobi<R>), grid_of(g), dim3(TX, TY), 0, s, g, b, u, out, omega, zero_guess ? 1 : 0);
}
template <typename R>
void launch_rb_colour(const Grid<R> &g, const cplx<R> *b, cplx<R> *u, R omega, int colour, bool zero_guess,
                      hipStream_t s) {
  launch_k((k_rb_colour<R>), grid_of(g), dim3(TX, TY), 0, s, g, b, u, omega, colour, zero_guess ? 1 : 0);
}
template <typename R>
void launch_restrict(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *rf, cplx<R> *rc, hipStream_t s) {
  launch_k((k_restrict<R>), grid_of(coarse), dim3(TX, TY), 0, s, fine, coarse, rf, rc);
}
template <typename R>
void launch_residual_restrict(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, const cplx<R> *u,
                              cplx<R> *rc, hipStream_t s) {
  launch_k((k_residual_restrict<R>), grid_of(coarse), dim3(TX, TY), 0, s, fine, coarse, b, u, rc);
}
template <typename R>
void launch_prolong_add(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *ec, cplx<R> *u, hipStream_t s) {
  launch_k((k_prolong_add<R>), grid_of(fine), dim3(TX, TY), 0, s, fine, coarse, ec, (const cplx<R> *)u, u);
}
template <typename R>
void launch_prolong_to(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *ec, const cplx<R> *u_in,
                       cplx<R> *u_out, hipStream_t s) {
  launch_k((k_prolong_add<R>), grid_of(fine), dim3(TX, TY), 0, s, fine, coarse, ec, u_in, u_out);
}
template <typename R>
void launch_prolong_jacobi(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *ec, const cplx<R> *b,
                           const cplx<R> *u, cplx<R> *out, R omega, hipStream_t s) {
  launch_k((k_prolong_jacobi<R>), grid_of(fine), dim3(TX, TY), 0, s, fine, coarse, ec, b, u, out, omega);
}
template <typename R>
void launch_coarse_solve(int nunk, const cplx<R> *minv, const int *unk, int n0, int n1, int n2, const cplx<R> *b,
                         cplx<R> *x, hipStream_t s, const RhsSet &rs) {
  if (multi_rhs(rs))
    launch_k((k_coarse_solve<R, true>), dim3(1, rs.count), dim3(1024), 0, s, nunk, minv, unk, n0, n1, n2, b, x, rs);
  else
    launch_k((k_coarse_solve<R, false>), dim3(1), dim3(1024), 0, s, nunk, minv, unk, n0, n1, n2, b, x, rs);
}
template <typename R, typename RI>
void launch_apply_dot(const Grid<R> &g, const cplx<RI> *x, cplx<R> *y, const cplx<R> *d0, int mode,
                      cplx<double> *partials, BicgScalars *S, hipStream_t s, const RhsSet &rs) {
  // one block per 64 x 4 tile while the partials (two per block) fit the
  // reduction buffer (kRedBlocks x (kMaxRestart + 2) entries); batched
  // launches (2D only) give every right-hand side kRhsPartials of them
  if (g.n2 == 1) {
    constexpr int sy = strip_rows<R, 1>();
    int tx, tiles, nb;
    strip_grid(g, sy, &tx, &tiles, &nb, rs.count > 1);
    const dim3 grid(nb, rs.count);
    const bool mr = multi_rhs(rs);
    if (mode == kBicgAlpha && mr)
      launch_k((k_apply2d<R, RI, R, kBicgAlpha, sy, true>), grid, dim3(256), 0, s, g, x, y, d0, partials, tx, tiles,
               rs);
    else if (mode == kBicgAlpha)
      launch_k((k_apply2d<R, RI, R, kBicgAlpha, sy>), grid, dim3(256), 0, s, g, x, y, d0, partials, tx, tiles, rs);
    else if (mr)
      launch_k((k_apply2d<R, RI, R, kBicgOmega, sy, true>), grid, dim3(256), 0, s, g, x, y, d0, partials, tx, tiles,
               rs);
    else
      launch_k((k_apply2d<R, RI, R, kBicgOmega, sy>), grid, dim3(256), 0, s, g, x, y, d0, partials, tx, tiles, rs);
    launch_bicg_final(partials, nb, mode == kBicgAlpha ? 1 : 2, S, mode, s, rs);
    return;
  }
  const int ntiles = ((g.n0 + TX - 1) / TX) * ((g.n1 + TY - 1) / TY) * g.n2;
  const int nb = ntiles < kRedBlocks ? ntiles : kRedBlocks;
  launch_k((k_apply_dot<R, RI>), dim3(nb), dim3(256), 0, s, g, x, y, d0, mode, partials, S);
  launch_bicg_final(partials, nb, mode == kBicgAlpha ? 1 : 2, S, mode, s);
}

template <typename R>
void launch_inject_k2(int n0, int n1, int n2, const double *k2_fine, int f0, int f1, R *k2_coarse, hipStream_t s) {
  int stride = (f0 - 1) / (n0 - 1);
  launch_k((k_inject_k2<R>), dim3((n0 + 255) / 256, n1, n2), dim3(256), 0, s, n0, n1, n2, k2_fine, f0, f1,
                     stride, k2_coarse);
}

#define ECS_INST_MG(R)                                                                                          \
  template void launch_residual<R>(const Grid<R> &, const cplx<R> *, const cplx<R> *, cplx<R> *, hipStream_t);  \
  template void launch_jacobi<R>(const Grid<R> &, const cplx<R> *, const cplx<R> *, cplx<R> *, R, bool,          \
                                 hipStream_t);                                                                  \
  template void launch_rb_colour<R>(const Grid<R> &, const cplx<R> *, cplx<R> *, R, int, bool, hipStream_t);     \
  template void launch_restrict<R>(const Grid<R> &, const Grid<R> &, const cplx<R> *, cplx<R> *, hipStream_t);   \
  template void launch_residual_restrict<R>(const Grid<R> &, const Grid<R> &, const cplx<R> *, const cplx<R> *,  \
                                            cplx<R> *, hipStream_t);                                            \
  template void launch_prolong_add<R>(const Grid<R> &, const Grid<R> &, const cplx<R> *, cplx<R> *,              \
                                      hipStream_t);                                                             \
  template void launch_prolong_jacobi<R>(const Grid<R> &, const Grid<R> &, const cplx<R> *, const cplx<R> *,      \
                                         const cplx<R> *, cplx<R> *, R, hipStream_t);                           \
  template void launch_prolong_to<R>(const Grid<R> &, const Grid<R> &, const cplx<R> *, const cplx<R> *,         \
                                     cplx<R> *, hipStream_t);                                                   \
  template void launch_coarse_solve<R>(int, const cplx<R> *, const int *, int, int, int, const cplx<R> *,      \
                                       cplx<R> *, hipStream_t, const RhsSet &);                                 \
  template void launch_inject_k2<R>(int, int, int, const double *, int, int, R *, hipStream_t);

ECS_INST_MG(double)
ECS_INST_MG(float)

template void launch_apply_dot<double, double>(const Grid<double> &, const cplx<double> *, cplx<double> *,
                                               const cplx<double> *, int, cplx<double> *, BicgScalars *, hipStream_t,
                                               const RhsSet &);
template void launch_apply_dot<double, float>(const Grid<double> &, const cplx<float> *, cplx<double> *,
                                              const cplx<double> *, int, cplx<double> *, BicgScalars *, hipStream_t,
                                              const RhsSet &);
template void launch_apply_dot<float, float>(const Grid<float> &, const cplx<float> *, cplx<float> *,
                                             const cplx<float> *, int, cplx<double> *, BicgScalars *, hipStream_t,
                                             const RhsSet &);
template void launch_apply<double, double, double>(const Grid<double> &, const cplx<double> *, cplx<double> *,
                                                   hipStream_t);
template void launch_apply<double, float, double>(const Grid<double> &, const cplx<float> *, cplx<double> *,
                                                  hipStream_t);
template void launch_apply<float, float, float>(const Grid<float> &, const cplx<float> *, cplx<float> *,
                                                hipStream_t);

}  // namespace ecs
