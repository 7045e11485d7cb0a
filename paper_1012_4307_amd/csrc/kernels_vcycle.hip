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
// thousand nodes a launch per level costs more than the work, so the down
// passes, the dense coarsest solve and the up passes of every level from the
// tail's first level to the coarsest run in one launch, phases separated by
// workgroup barriers.  Every level vector of the tail lives in LDS (at most
// kTailCap nodes over all tail levels): global memory is touched once at the
// start (the first level's right-hand side, the 1D weights and k^2 of all
// levels) and once at the end (the first level's result).
// Per level k (nodes [noff[k], noff[k+1]) of the LDS vectors):
//   b  right-hand side (the restricted residual of the level above)
//   t  pre-smoothed iterate
//   w  residual on the way down, corrected and post-smoothed iterate on the way up
//   d  inverse diagonal
constexpr int TT = 1024;  // tail threads
constexpr int TW = 128;   // LDS weights per axis and kind (>= sum of the tail level sizes)

template <typename R>
struct TailLds {
  cplx<R> xm[TW + 1], xp[TW + 1], ym[TW + 1], yp[TW + 1];  // + a spare slot
  cplx<R> b[kTailCap], t[kTailCap], w[kTailCap], d[kTailCap];
  cplx<R> mi[kTailMinv + 1];  // the coarsest inverse (transposed) when it fits, and a spare slot
};

// rows of the dense coarsest solve: tpr lanes per row, partial sums combined
// across the row's lanes; the interior unknowns are the interior nodes in
// row-major order
template <typename R, typename M>
__device__ __forceinline__ void tail_dense(int nu, int tpr, const M *mi, const cplx<R> *b, cplx<R> *x, int n0) {
  const int tid = threadIdx.x, ni = n0 - 2, rows_per_pass = TT / tpr;
  for (int r0 = 0; r0 < nu; r0 += rows_per_pass) {
    const int rr = r0 + tid / tpr;
    cplx<R> acc = zero_c<R>();
    if (rr < nu) {
#pragma unroll 4
      for (int c = tid % tpr; c < nu; c += tpr)
        acc = acc + mi[(int64_t)c * nu + rr] * b[(c / ni + 1) * n0 + c % ni + 1];
    }
    for (int m = tpr >> 1; m >= 1; m >>= 1) {
      acc.re += __shfl_xor(acc.re, m, 64);
      acc.im += __shfl_xor(acc.im, m, 64);
    }
    if (rr < nu && tid % tpr == 0) x[(rr / ni + 1) * n0 + rr % ni + 1] = acc;
  }
}

template <typename R>
__global__ __launch_bounds__(TT) void k_tail(TailArgs<R> a) {
  __shared__ TailLds<R> S;
  const int tid = threadIdx.x;
  const R om = a.omega, om1 = R(1) - a.omega;
  const int last = a.nl - 1;
  const bool minv_lds = a.nunk * a.nunk <= kTailMinv;

  // setup, one memory round trip: the 1D weights of every level into LDS, the
  // inverse diagonal of every node of every level, the first level's
  // right-hand side and its zero-guess red relaxation, the coarsest inverse.
  // Waves never straddle levels (per-level ranges padded to 64 lanes), so a
  // wave's level is uniform and the kernel arguments are indexed uniformly.
  // Loads use clamped (always valid) indexes and are issued before any use.
  {
    constexpr int kSlots = (kTailCap + kTailMaxLevels * 63 + TT - 1) / TT;
    // weights: wave k (k < nl) loads level k's, lane = node index
    const int kw = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool wl = kw < a.nl;
    const Grid<R> &gw = a.g[wl ? kw : 0];
    const int ln = tid & 63;
    const int q0 = ln < gw.n0 ? ln : gw.n0 - 1, q1 = ln < gw.n1 ? ln : gw.n1 - 1;
    const cplx<R> wxm = gw.cm0[q0], wxp = gw.cp0[q0], wym = gw.cm1[q1], wyp = gw.cp1[q1];
    // nodes: slot sl of thread tid is padded index P = tid + sl TT
    cplx<R> cxm[kSlots], cxp[kSlots], cym[kSlots], cyp[kSlots], bv[kSlots];
    R kv[kSlots];
    int lv[kSlots], pv[kSlots];
#pragma unroll
    for (int sl = 0; sl < kSlots; sl++) {
      const int P = tid + sl * TT;
      int k = 0;
      for (int q = 1; q < a.nl; q++) k = P >= a.poff[q] ? q : k;
      k = __builtin_amdgcn_readfirstlane(k);
      const Grid<R> &g = a.g[k];
      const int nn = g.n0 * g.n1;
      const int p0 = P - a.poff[k], p = p0 < nn ? p0 : nn - 1;
      const int i = p % g.n0, j = p / g.n0;
      lv[sl] = P < a.poff[a.nl] && p0 < nn ? k : -1;
      pv[sl] = p;
      cxm[sl] = g.cm0[i];
      cxp[sl] = g.cp0[i];
      cym[sl] = g.cm1[j];
      cyp[sl] = g.cp1[j];
      kv[sl] = g.k2[p];
      bv[sl] = a.b0[k == 0 ? p : 0];
    }
    constexpr int kMiSlots = (kTailMinv + TT - 1) / TT;
    const int nmi = a.nunk * a.nunk;
    cplx<R> mv[kMiSlots];
#pragma unroll
    for (int m = 0; m < kMiSlots; m++) {
      const int q2 = tid + m * TT;
      mv[m] = a.minvT[minv_lds && q2 < nmi ? q2 : 0];
    }
    // unconditional stores (unused entries to a spare slot) keep the loads
    // above ahead of every wait
#pragma unroll
    for (int m = 0; m < kMiSlots; m++) {
      const int q2 = tid + m * TT;
      S.mi[minv_lds && q2 < nmi ? q2 : kTailMinv] = mv[m];
    }
    const int wx = wl && ln < gw.n0 ? a.woff[kw] + ln : TW, wy = wl && ln < gw.n1 ? a.woff[kw] + ln : TW;
    S.xm[wx] = wxm;
    S.xp[wx] = wxp;
    S.ym[wy] = wym;
    S.yp[wy] = wyp;
#pragma unroll
    for (int sl = 0; sl < kSlots; sl++) {
      const int k = lv[sl];
      if (k < 0) continue;
      const int kk = __builtin_amdgcn_readfirstlane(k < 0 ? 0 : k);
      const Grid<R> &g = a.g[kk];
      const int p = pv[sl], i = p % g.n0, j = p / g.n0, P = a.noff[kk] + p;
      const bool in = i >= 1 && i <= g.n0 - 2 && j >= 1 && j <= g.n1 - 2;
      const cplx<R> dv = in ? inv_c(cxm[sl] + cxp[sl] + cym[sl] + cyp[sl] + (kv[sl] * g.beta + g.c)) : zero_c<R>();
      S.d[P] = dv;
      if (kk == 0) {
        const cplx<R> b = in ? bv[sl] : zero_c<R>();
        S.b[P] = b;
        S.t[P] = (in && ((i + j) & 1) == 0) ? om * (b * dv) : zero_c<R>();
      }
    }
  }
  __syncthreads();

  // down: black relaxation, red residual, restriction (which also performs
  // the next level's zero-guess red relaxation on the nodes it produces)
  for (int k = 0; k < last; k++) {
    const Grid<R> &g = a.g[k];
    const int n0 = g.n0, n1 = g.n1, nn = n0 * n1, no = a.noff[k], wo = a.woff[k];
    const cplx<R> *xm = S.xm + wo, *xp = S.xp + wo, *ym = S.ym + wo, *yp = S.yp + wo;
    cplx<R> *b = S.b + no, *t = S.t + no, *w = S.w + no, *d = S.d + no;
    for (int p = tid; p < nn; p += TT) {
      const int i = p % n0, j = p / n0;
      if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && ((i + j) & 1) == 1) {
        const cplx<R> tb = b[p] + (xm[i] * t[p - 1] + xp[i] * t[p + 1] + ym[j] * t[p - n0] + yp[j] * t[p + n0]);
        t[p] = om * (tb * d[p]);
        w[p] = om1 * tb;  // black residual (1 - w)(b + o)
      }
    }
    __syncthreads();
    for (int p = tid; p < nn; p += TT) {
      const int i = p % n0, j = p / n0;
      const bool in = i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2;
      if (!in) w[p] = zero_c<R>();
      else if (((i + j) & 1) == 0)  // red residual (1 - w) b + o
        w[p] = om1 * b[p] + (xm[i] * t[p - 1] + xp[i] * t[p + 1] + ym[j] * t[p - n0] + yp[j] * t[p + n0]);
    }
    __syncthreads();
    const Grid<R> &gc = a.g[k + 1];
    const int c0 = gc.n0, nc = c0 * gc.n1, nco = a.noff[k + 1];
    for (int q = tid; q < nc; q += TT) {
      const int I = q % c0, J = q / c0;
      cplx<R> acc = zero_c<R>(), tv = zero_c<R>();
      if (I >= 1 && I <= c0 - 2 && J >= 1 && J <= gc.n1 - 2) {
        const cplx<R> *r0 = w + (2 * J) * n0 + 2 * I;
        acc = R(0.25) * r0[0] + R(0.125) * (r0[-1] + r0[1] + r0[-n0] + r0[n0]) +
              R(0.0625) * (r0[-n0 - 1] + r0[-n0 + 1] + r0[n0 - 1] + r0[n0 + 1]);
        if (((I + J) & 1) == 0) tv = om * (acc * S.d[nco + q]);
      }
      S.b[nco + q] = acc;
      S.t[nco + q] = tv;
    }
    __syncthreads();
  }

  // dense solve on the coarsest level
  {
    const Grid<R> &g = a.g[last];
    const int nn = g.n0 * g.n1, no = a.noff[last];
    for (int p = tid; p < nn; p += TT) S.w[no + p] = zero_c<R>();
    __syncthreads();
    if (minv_lds) tail_dense(a.nunk, a.tpr, S.mi, S.b + no, S.w + no, g.n0);
    else tail_dense(a.nunk, a.tpr, a.minvT, S.b + no, S.w + no, g.n0);
    __syncthreads();
  }

  // up: prolongation + correction, then the red-black post-sweep in place;
  // the first level's black sweep writes the result to global memory
  for (int k = last - 1; k >= 0; k--) {
    const Grid<R> &g = a.g[k];
    const int n0 = g.n0, n1 = g.n1, nn = n0 * n1, no = a.noff[k], wo = a.woff[k];
    const int c0 = a.g[k + 1].n0;
    const cplx<R> *xm = S.xm + wo, *xp = S.xp + wo, *ym = S.ym + wo, *yp = S.yp + wo;
    const cplx<R> *b = S.b + no, *t = S.t + no, *d = S.d + no, *e = S.w + a.noff[k + 1];
    cplx<R> *w = S.w + no;
    for (int p = tid; p < nn; p += TT) {
      const int i = p % n0, j = p / n0;
      cplx<R> v = zero_c<R>();
      if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
        const cplx<R> *e0 = e + (j >> 1) * c0 + (i >> 1);
        const cplx<R> e1 = (i & 1) ? e0[1] : zero_c<R>();
        const cplx<R> e2 = (j & 1) ? e0[c0] : zero_c<R>();
        const cplx<R> e3 = ((i & 1) && (j & 1)) ? e0[c0 + 1] : zero_c<R>();
        const R wx = (i & 1) ? R(0.5) : R(1), wy = (j & 1) ? R(0.5) : R(1);
        v = t[p] + (wx * wy) * (e0[0] + e1 + e2 + e3);
      }
      w[p] = v;
    }
    __syncthreads();
    for (int colour = 0; colour < 2; colour++) {
      for (int p = tid; p < nn; p += TT) {
        const int i = p % n0, j = p / n0;
        const bool upd = i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2 && ((i + j) & 1) == colour;
        cplx<R> v = w[p];
        if (upd) {
          const cplx<R> o = xm[i] * w[p - 1] + xp[i] * w[p + 1] + ym[j] * w[p - n0] + yp[j] * w[p + n0];
          v = om1 * v + om * ((b[p] + o) * d[p]);
          w[p] = v;
        }
        if (k == 0 && colour == 1) a.u0[p] = v;
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
