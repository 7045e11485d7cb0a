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
                                                cplx<R> *__restrict__ u_out, cplx<R> *__restrict__ rc, R omega,
                                                int tiles_x, int tiles) {
  constexpr int CX = 29;
  constexpr int WX = 2 * CX + 5;          // 63 used columns
  constexpr int WY = 2 * CY + 5;
  constexpr int RPW = (WY + 3) / 4;       // rows per wave
  __shared__ cplx<R> su[WY][64];          // relaxed iterate
  __shared__ cplx<R> sr[WY][64];          // residual
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tile = xcd_tile(tiles);
  if (tile < 0) return;
  const int I0 = (tile % tiles_x) * CX, J0 = (tile / tiles_x) * CY;
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
                                              cplx<R> *__restrict__ u_out, R omega, int tiles_x, int tiles) {
  constexpr int TX = 60;
  constexpr int WY = TY + 4;
  constexpr int RPW = (WY + 3) / 4;
  constexpr int CWX = TX / 2 + 3, CWY = TY / 2 + 3;
  __shared__ cplx<R> sv[WY][64];
  __shared__ cplx<R> se[CWY][CWX];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tile = xcd_tile(tiles);
  if (tile < 0) return;
  const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
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

// ----------------------------------------------------------------- tail
// The coarsest levels of the cycle in one workgroup: for grids of a few
// thousand nodes a kernel launch per phase costs more than the work, so the
// down passes, the dense coarsest solve and the up passes of every level from
// the tail's first level to the coarsest run in one launch, phases separated
// by workgroup barriers.  Level vectors live in global memory (L2-resident);
// the 1D weights of all tail levels are staged in LDS; every phase first
// gathers the operands of all of a thread's nodes (TS slots, unrolled) and
// only then computes, so one memory round trip is paid per phase.
// Level k of the tail: b[k] right-hand side, t[k] pre-smoothed iterate, u[k]
// result.
constexpr int TT = 1024;  // tail threads
constexpr int TS = 2;     // node slots per thread: tail levels have <= 2048 nodes
constexpr int TW = 128;   // LDS weights per axis and kind (sum of the tail level sizes)

template <typename R>
struct TailW {
  cplx<R> xm[TW], xp[TW], ym[TW], yp[TW];
};

template <typename R>
__global__ __launch_bounds__(TT) void k_tail(TailArgs<R> a) {
  __shared__ TailW<R> W;
  __shared__ int off[kTailMaxLevels];
  const int tid = threadIdx.x;
  const R om = a.omega, om1 = R(1) - a.omega;
  const int last = a.nl - 1;
  if (tid == 0) {
    int o = 0;
    for (int k = 0; k < a.nl; k++) {
      off[k] = o;
      o += a.g[k].n0 > a.g[k].n1 ? a.g[k].n0 : a.g[k].n1;
    }
  }
  __syncthreads();
  for (int k = 0; k < a.nl; k++) {
    const Grid<R> &g = a.g[k];
    for (int q = tid; q < g.n0; q += TT) {
      W.xm[off[k] + q] = g.cm0[q];
      W.xp[off[k] + q] = g.cp0[q];
    }
    for (int q = tid; q < g.n1; q += TT) {
      W.ym[off[k] + q] = g.cm1[q];
      W.yp[off[k] + q] = g.cp1[q];
    }
  }
  __syncthreads();

  // down: zero-guess red-black sweep, then the restricted residual
  for (int k = 0; k < last; k++) {
    const Grid<R> &g = a.g[k];
    const cplx<R> *xm = W.xm + off[k], *xp = W.xp + off[k], *ym = W.ym + off[k], *yp = W.yp + off[k];
    const cplx<R> *b = a.b[k];
    cplx<R> *t = a.t[k];
    const int n0 = g.n0, n1 = g.n1, nn = n0 * n1;
    cplx<R> bs[TS], is[TS];
#pragma unroll
    for (int s = 0; s < TS; s++) {
      const int p = tid + s * TT;
      bs[s] = zero_c<R>();
      is[s] = zero_c<R>();
      if (p < nn) {
        const int i = p % n0, j = p / n0;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
          bs[s] = b[p];
          is[s] = inv_c(xm[i] + xp[i] + ym[j] + yp[j] + (g.k2[p] * g.beta + g.c));
        }
      }
    }
#pragma unroll
    for (int s = 0; s < TS; s++) {
      const int p = tid + s * TT;
      if (p < nn) {
        const int i = p % n0, j = p / n0;
        t[p] = ((i + j) & 1) == 0 ? om * (bs[s] * is[s]) : zero_c<R>();
      }
    }
    __syncthreads();
    cplx<R> nb[TS][4];
#pragma unroll
    for (int s = 0; s < TS; s++) {
      const int p = tid + s * TT;
      if (p < nn) {
        const int i = p % n0, j = p / n0;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && ((i + j) & 1) == 1) {
          nb[s][0] = t[p - 1]; nb[s][1] = t[p + 1]; nb[s][2] = t[p - n0]; nb[s][3] = t[p + n0];
        }
      }
    }
    cplx<R> rs[TS];
#pragma unroll
    for (int s = 0; s < TS; s++) {
      const int p = tid + s * TT;
      rs[s] = zero_c<R>();
      if (p < nn) {
        const int i = p % n0, j = p / n0;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && ((i + j) & 1) == 1) {
          const cplx<R> tb = bs[s] + (xm[i] * nb[s][0] + xp[i] * nb[s][1] + ym[j] * nb[s][2] + yp[j] * nb[s][3]);
          t[p] = om * (tb * is[s]);
          rs[s] = om1 * tb;  // black residual
        }
      }
    }
    __syncthreads();
    // red residuals from the relaxed black neighbours; residual vector kept in
    // the tail's scratch u[k] (free until the up pass overwrites it)
    cplx<R> *r = a.u[k];
#pragma unroll
    for (int s = 0; s < TS; s++) {
      const int p = tid + s * TT;
      if (p < nn) {
        const int i = p % n0, j = p / n0;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && ((i + j) & 1) == 0) {
          nb[s][0] = t[p - 1]; nb[s][1] = t[p + 1]; nb[s][2] = t[p - n0]; nb[s][3] = t[p + n0];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < TS; s++) {
      const int p = tid + s * TT;
      if (p < nn) {
        const int i = p % n0, j = p / n0;
        const bool in = i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2;
        if (in && ((i + j) & 1) == 0)
          rs[s] = om1 * bs[s] + (xm[i] * nb[s][0] + xp[i] * nb[s][1] + ym[j] * nb[s][2] + yp[j] * nb[s][3]);
        r[p] = in ? rs[s] : zero_c<R>();
      }
    }
    __syncthreads();
    const Grid<R> &gc = a.g[k + 1];
    cplx<R> *bc = a.b[k + 1];
    const int nc = gc.n0 * gc.n1;
    for (int q = tid; q < nc; q += TT) {
      const int I = q % gc.n0, J = q / gc.n0;
      cplx<R> acc = zero_c<R>();
      if (I >= 1 && I <= gc.n0 - 2 && J >= 1 && J <= gc.n1 - 2) {
        const cplx<R> *c0 = r + (int64_t)(2 * J) * n0 + 2 * I;
        acc = R(0.25) * c0[0] + R(0.125) * (c0[-1] + c0[1] + c0[-n0] + c0[n0]) +
              R(0.0625) * (c0[-n0 - 1] + c0[-n0 + 1] + c0[n0 - 1] + c0[n0 + 1]);
      }
      bc[q] = acc;
    }
    __syncthreads();
  }
  // dense solve on the coarsest level (inverse stored transposed)
  {
    const Grid<R> &g = a.g[last];
    const int nn = g.n0 * g.n1;
    cplx<R> *x = a.u[last];
    const cplx<R> *bb = a.b[last];
    for (int p = tid; p < nn; p += TT) {
      const int i = p % g.n0, j = p / g.n0;
      if (i < 1 || i > g.n0 - 2 || j < 1 || j > g.n1 - 2) x[p] = zero_c<R>();
    }
    for (int rr = tid; rr < a.nunk; rr += TT) {
      cplx<R> acc = zero_c<R>();
#pragma unroll 8
      for (int c = 0; c < a.nunk; c++) acc = acc + a.minvT[(int64_t)c * a.nunk + rr] * bb[a.unk[c]];
      x[a.unk[rr]] = acc;
    }
    __syncthreads();
  }
  // up: prolongation + correction, then the red-black post-sweep in place
  for (int k = last - 1; k >= 0; k--) {
    const Grid<R> &g = a.g[k];
    const Grid<R> &gc = a.g[k + 1];
    const cplx<R> *xm = W.xm + off[k], *xp = W.xp + off[k], *ym = W.ym + off[k], *yp = W.yp + off[k];
    const cplx<R> *b = a.b[k];
    const cplx<R> *t = a.t[k];
    const cplx<R> *ec = a.u[k + 1];
    cplx<R> *u = a.u[k];
    const int n0 = g.n0, n1 = g.n1, nn = n0 * n1;
    cplx<R> vs[TS], bs[TS], is[TS], e4[TS][4];
#pragma unroll
    for (int s = 0; s < TS; s++) {
      const int p = tid + s * TT;
      vs[s] = zero_c<R>();
      bs[s] = zero_c<R>();
      is[s] = zero_c<R>();
      if (p < nn) {
        const int i = p % n0, j = p / n0;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
          const cplx<R> *e = ec + (int64_t)(j >> 1) * gc.n0 + (i >> 1);
          e4[s][0] = e[0];
          e4[s][1] = (i & 1) ? e[1] : zero_c<R>();
          e4[s][2] = (j & 1) ? e[gc.n0] : zero_c<R>();
          e4[s][3] = ((i & 1) && (j & 1)) ? e[gc.n0 + 1] : zero_c<R>();
          vs[s] = t[p];
          bs[s] = b[p];
          is[s] = inv_c(xm[i] + xp[i] + ym[j] + yp[j] + (g.k2[p] * g.beta + g.c));
        }
      }
    }
#pragma unroll
    for (int s = 0; s < TS; s++) {
      const int p = tid + s * TT;
      if (p < nn) {
        const int i = p % n0, j = p / n0;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
          const R wx = (i & 1) ? R(0.5) : R(1), wy = (j & 1) ? R(0.5) : R(1);
          vs[s] = vs[s] + (wx * wy) * (e4[s][0] + e4[s][1] + e4[s][2] + e4[s][3]);
        }
        u[p] = vs[s];
      }
    }
    __syncthreads();
    for (int colour = 0; colour < 2; colour++) {
      cplx<R> nb[TS][4];
#pragma unroll
      for (int s = 0; s < TS; s++) {
        const int p = tid + s * TT;
        if (p < nn) {
          const int i = p % n0, j = p / n0;
          if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && ((i + j) & 1) == colour) {
            nb[s][0] = u[p - 1]; nb[s][1] = u[p + 1]; nb[s][2] = u[p - n0]; nb[s][3] = u[p + n0];
          }
        }
      }
#pragma unroll
      for (int s = 0; s < TS; s++) {
        const int p = tid + s * TT;
        if (p < nn) {
          const int i = p % n0, j = p / n0;
          if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && ((i + j) & 1) == colour) {
            const cplx<R> o = xm[i] * nb[s][0] + xp[i] * nb[s][1] + ym[j] * nb[s][2] + yp[j] * nb[s][3];
            vs[s] = om1 * vs[s] + om * ((bs[s] + o) * is[s]);
            u[p] = vs[s];
          }
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace

// The tile height of the fused kernels is a launch parameter chosen by the
// host (autotuned per grid size and dtype): coarse rows per down block in
// {2, 4, 8, 16} (16 only in FP32, whose tile fits the LDS), fine rows per up
// block in {4, 8, 16, 32}.
template <typename R>
void launch_down_rb(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, cplx<R> *u, cplx<R> *rc, R omega,
                    int rows, hipStream_t s) {
  constexpr int CX = 29;
  const int tx = (coarse.n0 + CX - 1) / CX;
  const int tiles = tx * ((coarse.n1 + rows - 1) / rows);
  const dim3 grid(xcd_padded(tiles)), block(NT);
  switch (rows) {
    case 2: hipLaunchKernelGGL((k_down_rb<R, 2>), grid, block, 0, s, fine, coarse, b, u, rc, omega, tx, tiles); break;
    case 4: hipLaunchKernelGGL((k_down_rb<R, 4>), grid, block, 0, s, fine, coarse, b, u, rc, omega, tx, tiles); break;
    case 16:
      if constexpr (sizeof(R) == 4) {
        hipLaunchKernelGGL((k_down_rb<R, 16>), grid, block, 0, s, fine, coarse, b, u, rc, omega, tx, tiles);
        break;
      }
      [[fallthrough]];
    default: hipLaunchKernelGGL((k_down_rb<R, 8>), grid, block, 0, s, fine, coarse, b, u, rc, omega, tx, tiles); break;
  }
}

template <typename R>
void launch_up_rb(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, const cplx<R> *u_in,
                  const cplx<R> *ec, cplx<R> *u_out, R omega, int rows, hipStream_t s) {
  constexpr int TX = 60;
  const int tx = (fine.n0 + TX - 1) / TX;
  const int tiles = tx * ((fine.n1 + rows - 1) / rows);
  const dim3 grid(xcd_padded(tiles)), block(NT);
  switch (rows) {
    case 4: hipLaunchKernelGGL((k_up_rb<R, 4>), grid, block, 0, s, fine, coarse, b, u_in, ec, u_out, omega, tx, tiles); break;
    case 8: hipLaunchKernelGGL((k_up_rb<R, 8>), grid, block, 0, s, fine, coarse, b, u_in, ec, u_out, omega, tx, tiles); break;
    case 32: hipLaunchKernelGGL((k_up_rb<R, 32>), grid, block, 0, s, fine, coarse, b, u_in, ec, u_out, omega, tx, tiles); break;
    default: hipLaunchKernelGGL((k_up_rb<R, 16>), grid, block, 0, s, fine, coarse, b, u_in, ec, u_out, omega, tx, tiles); break;
  }
}

template <typename R>
void launch_tail(const TailArgs<R> &a, hipStream_t s) {
  hipLaunchKernelGGL((k_tail<R>), dim3(1), dim3(TT), 0, s, a);
}

template void launch_down_rb<double>(const Grid<double> &, const Grid<double> &, const cplx<double> *, cplx<double> *,
                                     cplx<double> *, double, int, hipStream_t);
template void launch_down_rb<float>(const Grid<float> &, const Grid<float> &, const cplx<float> *, cplx<float> *,
                                    cplx<float> *, float, int, hipStream_t);
template void launch_up_rb<double>(const Grid<double> &, const Grid<double> &, const cplx<double> *,
                                   const cplx<double> *, const cplx<double> *, cplx<double> *, double, int,
                                   hipStream_t);
template void launch_tail<double>(const TailArgs<double> &, hipStream_t);
template void launch_tail<float>(const TailArgs<float> &, hipStream_t);
template void launch_up_rb<float>(const Grid<float> &, const Grid<float> &, const cplx<float> *, const cplx<float> *,
                                  const cplx<float> *, cplx<float> *, float, int, hipStream_t);

}  // namespace ecs
