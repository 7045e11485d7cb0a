// kernels_vcycle.hip -- fused 2D kernels of the V(1,1) red-black cycle (the
// QD set-up of bin Zubair, Reps, Vanroose, Sec. 4.2: one red-black SOR sweep
// before and after the coarse-grid correction, full weighting, bilinear
// interpolation).  Each level is visited by exactly two kernels:
//
//   down: u = S_rb(0; b) (zero-guess sweep), rc = FW(b - M u)
//         reads b, k^2 once, writes u and the coarse residual
//   up:   v = u + P ec, u_out = S_rb(v; b) (post-sweep, out of place)
//         reads u, ec, b, k^2 once, writes u_out
//
// against four (pre-sweep, residual+FW, prolongation, post-sweep) in the
// generic path whose sweeps make two passes over the grid.  A block owns a tile
// of the fine grid; the values it needs around the tile (a red node depends on
// its black neighbours, a black node on the just-relaxed red ones, a residual
// on the relaxed neighbourhood, a restricted residual on 3x3 residuals) are
// recomputed redundantly from a halo staged in LDS, so tiles are independent
// and no grid-wide synchronisation is needed.  Rows are loaded with
// consecutive lanes on consecutive x (unit stride, interleaved complex).
#include "ecs_internal.h"

namespace ecs {

namespace {

constexpr int NT = 256;

template <typename R>
__device__ __forceinline__ cplx<R> zero_c() {
  return mk<R>(0, 0);
}

// ----------------------------------------------------------------- down
// Block tile: CX x CY coarse nodes starting at (I0, J0); owned fine nodes are
// [2 I0, 2 I0 + 2 CX) x [2 J0, 2 J0 + 2 CY).  Staged region: fine x in
// [2 I0 - 3, 2 I0 + 2 CX + 1], y likewise (halo 3 on the low side, 2 on the
// high side; the residual of the FW stencil at the tile's last coarse node
// reaches 2 I0 + 2 CX - 1, its relaxed neighbourhood 2 I0 + 2 CX, and the red
// values that feed it 2 I0 + 2 CX + 1).
template <typename R, int CX, int CY>
__global__ __launch_bounds__(NT) void k_down_rb(Grid<R> f, Grid<R> c, const cplx<R> *__restrict__ b,
                                                cplx<R> *__restrict__ u_out, cplx<R> *__restrict__ rc, R omega) {
  constexpr int WX = 2 * CX + 5, WY = 2 * CY + 5;
  constexpr int NR = WX * WY;
  __shared__ cplx<R> sb[NR];   // b, then the residual
  __shared__ cplx<R> sd[NR];   // diagonal of M
  __shared__ cplx<R> su[NR];   // relaxed iterate
  const int I0 = blockIdx.x * CX, J0 = blockIdx.y * CY;
  const int gx0 = 2 * I0 - 3, gy0 = 2 * J0 - 3;
  const int n0 = f.n0, n1 = f.n1;

  // stage b and the diagonal; mark the red iterate omega b / D
  for (int q = threadIdx.x; q < NR; q += NT) {
    const int lx = q % WX, ly = q / WX;
    const int i = gx0 + lx, j = gy0 + ly;
    cplx<R> bv = zero_c<R>(), dv = mk<R>(1, 0), uv = zero_c<R>();
    if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
      const int64_t p = (int64_t)j * n0 + i;
      bv = b[p];
      dv = f.cm0[i] + f.cp0[i] + f.cm1[j] + f.cp1[j] + (f.k2[p] * f.beta + f.c);
      if (((i + j) & 1) == 0) uv = omega * cdiv(bv, dv);
    }
    sb[q] = bv;
    sd[q] = dv;
    su[q] = uv;
  }
  __syncthreads();
  // black relaxation from the red values (zero guess: u_b = omega (b + offd) / D)
  for (int q = threadIdx.x; q < NR; q += NT) {
    const int lx = q % WX, ly = q / WX;
    const int i = gx0 + lx, j = gy0 + ly;
    if (lx < 1 || lx > WX - 2 || ly < 1 || ly > WY - 2) continue;
    if (i < 1 || i > n0 - 2 || j < 1 || j > n1 - 2 || ((i + j) & 1) == 0) continue;
    cplx<R> o = f.cm0[i] * su[q - 1] + f.cp0[i] * su[q + 1] + f.cm1[j] * su[q - WX] + f.cp1[j] * su[q + WX];
    su[q] = omega * cdiv(sb[q] + o, sd[q]);
  }
  __syncthreads();
  // residual r = b - M u on the interior (stored over b), 0 elsewhere; write u
  for (int q = threadIdx.x; q < NR; q += NT) {
    const int lx = q % WX, ly = q / WX;
    const int i = gx0 + lx, j = gy0 + ly;
    if (lx < 1 || lx > WX - 2 || ly < 1 || ly > WY - 2) continue;
    cplx<R> r = zero_c<R>();
    if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
      cplx<R> o = f.cm0[i] * su[q - 1] + f.cp0[i] * su[q + 1] + f.cm1[j] * su[q - WX] + f.cp1[j] * su[q + WX];
      r = sb[q] - (sd[q] * su[q] - o);
    }
    // owned fine nodes: local [3, 3 + 2 CX) x [3, 3 + 2 CY)
    if (lx >= 3 && lx < 3 + 2 * CX && ly >= 3 && ly < 3 + 2 * CY && i < n0 && j < n1)
      u_out[(int64_t)j * n0 + i] = su[q];
    sb[q] = r;  // each thread overwrites only its own node; other threads read su only
  }
  __syncthreads();
  // full weighting onto the owned coarse nodes
  for (int q = threadIdx.x; q < CX * CY; q += NT) {
    const int cx = q % CX, cy = q / CX;
    const int I = I0 + cx, J = J0 + cy;
    if (I >= c.n0 || J >= c.n1) continue;
    cplx<R> acc = zero_c<R>();
    if (I >= 1 && I <= c.n0 - 2 && J >= 1 && J <= c.n1 - 2) {
      const int lc = (3 + 2 * cy) * WX + (3 + 2 * cx);
      acc = R(0.25) * sb[lc] +
            R(0.125) * (sb[lc - 1] + sb[lc + 1] + sb[lc - WX] + sb[lc + WX]) +
            R(0.0625) * (sb[lc - WX - 1] + sb[lc - WX + 1] + sb[lc + WX - 1] + sb[lc + WX + 1]);
    }
    rc[(int64_t)J * c.n0 + I] = acc;
  }
}

// ------------------------------------------------------------------- up
// Block tile: TX x TY fine nodes at (x0, y0) with x0, y0 even.  Staged: the
// corrected iterate v = u + P ec on [x0 - 2, x0 + TX + 1] (halo 2: red nodes
// one outside the tile are relaxed, and read black neighbours two outside),
// b and D on the same region, the coarse correction under it.
template <typename R, int TX, int TY>
__global__ __launch_bounds__(NT) void k_up_rb(Grid<R> f, Grid<R> c, const cplx<R> *__restrict__ b,
                                              const cplx<R> *__restrict__ u_in, const cplx<R> *__restrict__ ec,
                                              cplx<R> *__restrict__ u_out, R omega) {
  constexpr int WX = TX + 4, WY = TY + 4;
  constexpr int NR = WX * WY;
  constexpr int CWX = TX / 2 + 3, CWY = TY / 2 + 3;
  __shared__ cplx<R> sv[NR];
  __shared__ cplx<R> sb[NR];
  __shared__ cplx<R> sd[NR];
  __shared__ cplx<R> se[CWX * CWY];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int gx0 = x0 - 2, gy0 = y0 - 2;
  const int cx0 = x0 / 2 - 1, cy0 = y0 / 2 - 1;  // coarse staging origin
  const int n0 = f.n0, n1 = f.n1;

  for (int q = threadIdx.x; q < CWX * CWY; q += NT) {
    const int I = cx0 + q % CWX, J = cy0 + q / CWX;
    se[q] = (I >= 0 && I < c.n0 && J >= 0 && J < c.n1) ? ec[(int64_t)J * c.n0 + I] : zero_c<R>();
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NR; q += NT) {
    const int lx = q % WX, ly = q / WX;
    const int i = gx0 + lx, j = gy0 + ly;
    cplx<R> v = zero_c<R>(), bv = zero_c<R>(), dv = mk<R>(1, 0);
    if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
      const int64_t p = (int64_t)j * n0 + i;
      // bilinear interpolation in index space from the staged coarse tile
      const int I = i >> 1, J = j >> 1;
      const int ci = I - cx0, cj = J - cy0;
      const cplx<R> *e = se + cj * CWX + ci;
      cplx<R> pe;
      if ((i & 1) == 0 && (j & 1) == 0) pe = e[0];
      else if ((j & 1) == 0) pe = R(0.5) * (e[0] + e[1]);
      else if ((i & 1) == 0) pe = R(0.5) * (e[0] + e[CWX]);
      else pe = R(0.25) * (e[0] + e[1] + e[CWX] + e[CWX + 1]);
      v = u_in[p] + pe;
      bv = b[p];
      dv = f.cm0[i] + f.cp0[i] + f.cm1[j] + f.cp1[j] + (f.k2[p] * f.beta + f.c);
    }
    sv[q] = v;
    sb[q] = bv;
    sd[q] = dv;
  }
  __syncthreads();
  // red relaxation on the tile plus a one-node ring
  for (int q = threadIdx.x; q < NR; q += NT) {
    const int lx = q % WX, ly = q / WX;
    const int i = gx0 + lx, j = gy0 + ly;
    if (lx < 1 || lx > WX - 2 || ly < 1 || ly > WY - 2) continue;
    if (i < 1 || i > n0 - 2 || j < 1 || j > n1 - 2 || ((i + j) & 1) != 0) continue;
    const cplx<R> u0 = sv[q];
    cplx<R> o = f.cm0[i] * sv[q - 1] + f.cp0[i] * sv[q + 1] + f.cm1[j] * sv[q - WX] + f.cp1[j] * sv[q + WX];
    cplx<R> res = sb[q] - (sd[q] * u0 - o);
    sv[q] = u0 + omega * cdiv(res, sd[q]);
  }
  __syncthreads();
  // black relaxation on the owned tile, then write every owned node
  for (int q = threadIdx.x; q < TX * TY; q += NT) {
    const int lx = 2 + q % TX, ly = 2 + q / TX;
    const int i = gx0 + lx, j = gy0 + ly;
    if (i >= n0 || j >= n1) continue;
    const int s = ly * WX + lx;
    cplx<R> out = sv[s];
    if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && ((i + j) & 1) == 1) {
      cplx<R> o = f.cm0[i] * sv[s - 1] + f.cp0[i] * sv[s + 1] + f.cm1[j] * sv[s - WX] + f.cp1[j] * sv[s + WX];
      cplx<R> res = sb[s] - (sd[s] * out - o);
      out = out + omega * cdiv(res, sd[s]);
    }
    u_out[(int64_t)j * n0 + i] = out;
  }
}

// tile shapes: LDS per block stays near 32 KB (FP64) so several blocks share a CU
template <typename R>
struct Tiles;
template <>
struct Tiles<double> {
  static constexpr int DCX = 16, DCY = 8;   // down: 32 x 16 fine nodes per block
  static constexpr int UTX = 32, UTY = 16;  // up
};
template <>
struct Tiles<float> {
  static constexpr int DCX = 32, DCY = 8;   // down: 64 x 16 fine nodes per block
  static constexpr int UTX = 64, UTY = 16;
};

}  // namespace

template <typename R>
void launch_down_rb(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, cplx<R> *u, cplx<R> *rc, R omega,
                    hipStream_t s) {
  constexpr int CX = Tiles<R>::DCX, CY = Tiles<R>::DCY;
  dim3 grid((coarse.n0 + CX - 1) / CX, (coarse.n1 + CY - 1) / CY);
  hipLaunchKernelGGL((k_down_rb<R, CX, CY>), grid, dim3(NT), 0, s, fine, coarse, b, u, rc, omega);
}

template <typename R>
void launch_up_rb(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, const cplx<R> *u_in,
                  const cplx<R> *ec, cplx<R> *u_out, R omega, hipStream_t s) {
  constexpr int TX = Tiles<R>::UTX, TY = Tiles<R>::UTY;
  dim3 grid((fine.n0 + TX - 1) / TX, (fine.n1 + TY - 1) / TY);
  hipLaunchKernelGGL((k_up_rb<R, TX, TY>), grid, dim3(NT), 0, s, fine, coarse, b, u_in, ec, u_out, omega);
}

template void launch_down_rb<double>(const Grid<double> &, const Grid<double> &, const cplx<double> *, cplx<double> *,
                                     cplx<double> *, double, hipStream_t);
template void launch_down_rb<float>(const Grid<float> &, const Grid<float> &, const cplx<float> *, cplx<float> *,
                                    cplx<float> *, float, hipStream_t);
template void launch_up_rb<double>(const Grid<double> &, const Grid<double> &, const cplx<double> *,
                                   const cplx<double> *, const cplx<double> *, cplx<double> *, double, hipStream_t);
template void launch_up_rb<float>(const Grid<float> &, const Grid<float> &, const cplx<float> *, const cplx<float> *,
                                  const cplx<float> *, cplx<float> *, float, hipStream_t);

}  // namespace ecs
