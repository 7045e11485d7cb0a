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

// Both kernels first issue every global load of the block (register arrays
// of PER entries per thread, unrolled, so all are in flight together) and
// stage the tile's 1D weights in LDS.  A thread keeps the values of its own
// nodes (b, the inverse diagonal, its iterate) in registers across the phases;
// only the iterate and the residual, which neighbours read, go through LDS.
//
// With M u = D u - o(u), o the off-diagonal part, a red-black sweep relaxes
// u_p <- (1 - w) u_p + w (b_p + o_p) / D_p.  From a zero guess the residual
// after the sweep is (1 - w) b + o at red nodes (o from the relaxed black
// neighbours) and (1 - w)(b + o) at black nodes (o from the red ones), so the
// diagonal is never multiplied back.

template <typename R>
__device__ __forceinline__ cplx<R> inv_c(cplx<R> d) {
  const R s = R(1) / abs2(d);
  return mk<R>(d.re * s, -d.im * s);
}

// ----------------------------------------------------------------- down
// One lane per tile column (64 lanes = the tile width, so the x index, the x
// weights and the x bounds test are per-thread constants), the 4 waves of the
// block take every fourth tile row.  Block tile: CX = 29 coarse columns x CY
// coarse rows from (I0, J0); owned fine nodes [2 I0, 2 I0 + 58) x
// [2 J0, 2 J0 + 2 CY).  Staged fine region: columns 2 I0 - 3 + [0, 63) (lane
// 63 idles), rows 2 J0 - 3 + [0, 2 CY + 5): halo 3 below, 2 above, because
// the FW stencil of the tile's coarse nodes reads residuals one node out, a
// residual reads the relaxed iterate one further out, and a relaxed black node
// reads red values one further still.
template <typename R, int CY>
__global__ __launch_bounds__(NT) void k_down_rb(Grid<R> f, Grid<R> c, const cplx<R> *__restrict__ b,
                                                cplx<R> *__restrict__ u_out, cplx<R> *__restrict__ rc, R omega) {
  constexpr int CX = 29;
  constexpr int WX = 2 * CX + 5;          // 63 used columns
  constexpr int WY = 2 * CY + 5;
  constexpr int RPW = (WY + 3) / 4;       // rows per wave
  __shared__ cplx<R> su[WY][64];          // relaxed iterate
  __shared__ cplx<R> sr[WY][64];          // residual
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int I0 = blockIdx.x * CX, J0 = blockIdx.y * CY;
  const int gx0 = 2 * I0 - 3, gy0 = 2 * J0 - 3;
  const int n0 = f.n0, n1 = f.n1;
  const R om1 = R(1) - omega;
  const int i = gx0 + lane;
  const bool xin = lane < WX && i >= 1 && i <= n0 - 2;
  const cplx<R> cxm = xin ? f.cm0[i] : zero_c<R>();
  const cplx<R> cxp = xin ? f.cp0[i] : zero_c<R>();

  cplx<R> bv[RPW], iv[RPW], cym[RPW], cyp[RPW];
  R kv[RPW];
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    const int j = gy0 + ly;
    const bool yin = ly < WY && j >= 1 && j <= n1 - 2;
    bv[r] = zero_c<R>();
    kv[r] = R(0);
    cym[r] = yin ? f.cm1[j] : zero_c<R>();
    cyp[r] = yin ? f.cp1[j] : zero_c<R>();
    if (xin && yin) {
      const int64_t p = (int64_t)j * n0 + i;
      bv[r] = b[p];
      kv[r] = f.k2[p];
    }
  }
  // inverse diagonal; red iterate omega b / D (zero guess), black 0
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    if (ly >= WY) break;
    const int j = gy0 + ly;
    const bool in = xin && j >= 1 && j <= n1 - 2;
    iv[r] = in ? inv_c(cxm + cxp + cym[r] + cyp[r] + (kv[r] * f.beta + f.c)) : zero_c<R>();
    su[ly][lane] = (in && ((i + j) & 1) == 0) ? omega * (bv[r] * iv[r]) : zero_c<R>();
  }
  __syncthreads();
  // black relaxation; black residual (1 - w)(b + o)
  const bool xmid = lane >= 1 && lane <= WX - 2;
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    if (ly >= WY) break;
    const int j = gy0 + ly;
    if (!xmid || ly < 1 || ly > WY - 2 || !xin || j < 1 || j > n1 - 2 || ((i + j) & 1) == 0) continue;
    const cplx<R> tb = bv[r] + (cxm * su[ly][lane - 1] + cxp * su[ly][lane + 1] + cym[r] * su[ly - 1][lane] +
                                cyp[r] * su[ly + 1][lane]);
    su[ly][lane] = omega * (tb * iv[r]);
    sr[ly][lane] = om1 * tb;
  }
  __syncthreads();
  // red residual (1 - w) b + o, zero off the interior; write the owned iterate
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    if (ly >= WY) break;
    const int j = gy0 + ly;
    if (!xmid || ly < 1 || ly > WY - 2) continue;
    const bool in = xin && j >= 1 && j <= n1 - 2;
    if (!in) {
      sr[ly][lane] = zero_c<R>();
    } else if (((i + j) & 1) == 0) {
      sr[ly][lane] = om1 * bv[r] + (cxm * su[ly][lane - 1] + cxp * su[ly][lane + 1] + cym[r] * su[ly - 1][lane] +
                                    cyp[r] * su[ly + 1][lane]);
    }
    if (lane >= 3 && lane < 3 + 2 * CX && ly >= 3 && ly < 3 + 2 * CY && i < n0 && j < n1)
      u_out[(int64_t)j * n0 + i] = su[ly][lane];
  }
  __syncthreads();
  // full weighting onto the owned coarse nodes: lane = coarse column
  if (lane < CX) {
    const int I = I0 + lane;
    for (int cy = wv; cy < CY; cy += 4) {
      const int J = J0 + cy;
      if (I >= c.n0 || J >= c.n1) continue;
      cplx<R> acc = zero_c<R>();
      if (I >= 1 && I <= c.n0 - 2 && J >= 1 && J <= c.n1 - 2) {
        const int x = 3 + 2 * lane, y = 3 + 2 * cy;
        acc = R(0.25) * sr[y][x] + R(0.125) * (sr[y][x - 1] + sr[y][x + 1] + sr[y - 1][x] + sr[y + 1][x]) +
              R(0.0625) * (sr[y - 1][x - 1] + sr[y - 1][x + 1] + sr[y + 1][x - 1] + sr[y + 1][x + 1]);
      }
      rc[(int64_t)J * c.n0 + I] = acc;
    }
  }
}

// ------------------------------------------------------------------- up
// Same layout: lane = tile column.  Block tile: 60 x TY fine nodes at
// (x0, y0), both even; staged fine region: columns x0 - 2 + [0, 64), rows
// y0 - 2 + [0, TY + 4) (halo 2: red nodes one outside the tile are relaxed
// and read black neighbours two outside), and the coarse correction under it.
template <typename R, int TY>
__global__ __launch_bounds__(NT) void k_up_rb(Grid<R> f, Grid<R> c, const cplx<R> *__restrict__ b,
                                              const cplx<R> *__restrict__ u_in, const cplx<R> *__restrict__ ec,
                                              cplx<R> *__restrict__ u_out, R omega) {
  constexpr int TX = 60;
  constexpr int WY = TY + 4;
  constexpr int RPW = (WY + 3) / 4;
  constexpr int CWX = TX / 2 + 3, CWY = TY / 2 + 3;
  __shared__ cplx<R> sv[WY][64];
  __shared__ cplx<R> se[CWY][CWX];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int gx0 = x0 - 2, gy0 = y0 - 2;
  const int cx0 = x0 / 2 - 1, cy0 = y0 / 2 - 1;  // coarse staging origin
  const int n0 = f.n0, n1 = f.n1;
  const R om1 = R(1) - omega;
  const int i = gx0 + lane;
  const bool xin = i >= 1 && i <= n0 - 2;
  const cplx<R> cxm = xin ? f.cm0[i] : zero_c<R>();
  const cplx<R> cxp = xin ? f.cp0[i] : zero_c<R>();

  cplx<R> vv[RPW], bv[RPW], iv[RPW], cym[RPW], cyp[RPW];
  R kv[RPW];
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    const int j = gy0 + ly;
    const bool yin = ly < WY && j >= 1 && j <= n1 - 2;
    vv[r] = zero_c<R>();
    bv[r] = zero_c<R>();
    kv[r] = R(0);
    cym[r] = yin ? f.cm1[j] : zero_c<R>();
    cyp[r] = yin ? f.cp1[j] : zero_c<R>();
    if (xin && yin) {
      const int64_t p = (int64_t)j * n0 + i;
      vv[r] = u_in[p];
      bv[r] = b[p];
      kv[r] = f.k2[p];
    }
  }
  if (lane < CWX) {
    const int I = cx0 + lane;
    for (int cy = wv; cy < CWY; cy += 4) {
      const int J = cy0 + cy;
      se[cy][lane] = (I >= 0 && I < c.n0 && J >= 0 && J < c.n1) ? ec[(int64_t)J * c.n0 + I] : zero_c<R>();
    }
  }
  __syncthreads();
  // v = u + P ec (bilinear in index space) and the inverse diagonal
  const int ci = (i >> 1) - cx0;
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    if (ly >= WY) break;
    const int j = gy0 + ly;
    const bool in = xin && j >= 1 && j <= n1 - 2;
    iv[r] = zero_c<R>();
    if (in) {
      const int cj = (j >> 1) - cy0;
      cplx<R> pe;
      if ((i & 1) == 0 && (j & 1) == 0) pe = se[cj][ci];
      else if ((j & 1) == 0) pe = R(0.5) * (se[cj][ci] + se[cj][ci + 1]);
      else if ((i & 1) == 0) pe = R(0.5) * (se[cj][ci] + se[cj + 1][ci]);
      else pe = R(0.25) * (se[cj][ci] + se[cj][ci + 1] + se[cj + 1][ci] + se[cj + 1][ci + 1]);
      vv[r] = vv[r] + pe;
      iv[r] = inv_c(cxm + cxp + cym[r] + cyp[r] + (kv[r] * f.beta + f.c));
    }
    sv[ly][lane] = vv[r];
  }
  __syncthreads();
  // red relaxation on the tile plus a one-node ring
  const bool xmid = lane >= 1 && lane <= 62;
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    if (ly >= WY) break;
    const int j = gy0 + ly;
    if (!xmid || ly < 1 || ly > WY - 2 || !xin || j < 1 || j > n1 - 2 || ((i + j) & 1) != 0) continue;
    const cplx<R> o = cxm * sv[ly][lane - 1] + cxp * sv[ly][lane + 1] + cym[r] * sv[ly - 1][lane] +
                      cyp[r] * sv[ly + 1][lane];
    vv[r] = om1 * vv[r] + omega * ((bv[r] + o) * iv[r]);
    sv[ly][lane] = vv[r];
  }
  __syncthreads();
  // black relaxation on the owned tile; write every owned node
  const bool xown = lane >= 2 && lane < TX + 2 && i < n0;
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    if (ly >= WY) break;
    const int j = gy0 + ly;
    if (!xown || ly < 2 || ly >= TY + 2 || j >= n1) continue;
    cplx<R> out = vv[r];
    if (xin && j >= 1 && j <= n1 - 2 && ((i + j) & 1) == 1) {
      const cplx<R> o = cxm * sv[ly][lane - 1] + cxp * sv[ly][lane + 1] + cym[r] * sv[ly - 1][lane] +
                        cyp[r] * sv[ly + 1][lane];
      out = om1 * out + omega * ((bv[r] + o) * iv[r]);
    }
    u_out[(int64_t)j * n0 + i] = out;
  }
}

// tile heights (coarse rows for down, fine rows for up)
template <typename R>
struct Tiles;
template <>
struct Tiles<double> {
  static constexpr int DCY = 8, UTY = 16;
};
template <>
struct Tiles<float> {
  static constexpr int DCY = 16, UTY = 32;
};

}  // namespace

template <typename R>
void launch_down_rb(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, cplx<R> *u, cplx<R> *rc, R omega,
                    hipStream_t s) {
  constexpr int CX = 29, CY = Tiles<R>::DCY;
  dim3 grid((coarse.n0 + CX - 1) / CX, (coarse.n1 + CY - 1) / CY);
  hipLaunchKernelGGL((k_down_rb<R, CY>), grid, dim3(NT), 0, s, fine, coarse, b, u, rc, omega);
}

template <typename R>
void launch_up_rb(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, const cplx<R> *u_in,
                  const cplx<R> *ec, cplx<R> *u_out, R omega, hipStream_t s) {
  constexpr int TX = 60, TY = Tiles<R>::UTY;
  dim3 grid((fine.n0 + TX - 1) / TX, (fine.n1 + TY - 1) / TY);
  hipLaunchKernelGGL((k_up_rb<R, TY>), grid, dim3(NT), 0, s, fine, coarse, b, u_in, ec, u_out, omega);
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
