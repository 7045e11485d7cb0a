// kernels_vpair.hip -- two levels of the 2D V(1,1) red-black cycle (Sec. 4.2:
// one red-black SOR sweep before and after the coarse-grid correction, full
// weighting, bilinear interpolation) in one kernel, for the small levels of
// the hierarchy.  There a level's pass is a few microseconds of latency
// (launch, one memory round trip, a handful of barriers) around very little
// work, so fusing two levels removes a launch and a round trip per direction.
//
//   down2: level l    zero-guess sweep, residual, FW        -> b_{l+1}
//          level l+1  zero-guess sweep, residual, FW        -> b_{l+2}
//   up2:   level l+1  v = t + P e_{l+2}, red-black post-sweep -> u_{l+1}
//          level l    v = t + P u_{l+1}, red-black post-sweep -> u_l
//
// A block owns an output tile and recomputes every value its tile needs
// around it (the same halo reasoning as the one-level kernels, applied twice),
// so blocks are independent.  All region vectors live in LDS in natural
// row-major layout; a phase loops over the region with the row index taken
// from a float reciprocal (exact here), and colour phases loop over node
// pairs (columns 2h, 2h + 1 of a row: one red, one black).  Intermediate
// vectors that no later kernel reads (u_{l+1} in up2) never reach global
// memory; b_{l+1}, t_l and t_{l+1} are written for the owned nodes because
// the up pass reads them.
#include "ecs_internal.h"

namespace ecs {

namespace {

constexpr int NP = 512;  // threads per block

template <typename R>
__device__ __forceinline__ cplx<R> zc() {
  return mk<R>(0, 0);
}

template <typename R>
__device__ __forceinline__ cplx<R> inv_p(cplx<R> d) {
  R s;
  if constexpr (sizeof(R) == 4) s = __builtin_amdgcn_rcpf(abs2(d));
  else s = R(1) / abs2(d);
  return mk<R>(d.re * s, -d.im * s);
}

// (x, y) of flattened index q in a region of width w (float reciprocal: the
// rounding error is far below the half-cell margin for these sizes)
__device__ __forceinline__ void xy_of(int q, int w, float invw, int &x, int &y) {
  y = (int)(((float)q + 0.5f) * invw);
  x = q - y * w;
}

// A staged region of one level: origin (ox, oy) in the level's node indices,
// w x h nodes, vectors in LDS with row stride w.
template <typename R>
struct Region {
  int ox, oy, w, h;
  float invw, invh2;  // 1 / w, 1 / ceil(w / 2)
  // the level's 1D weights over the region's columns and rows, in LDS from
  // wt: xm at [0, w), xp at [w, 2w), ym at [2w, 2w + h), yp after them.  One
  // base and integer offsets (four separate pointers, selected between at
  // run time, were kept in scratch memory and read through flat accesses).
  cplx<R> *wt;
  __device__ __forceinline__ cplx<R> xm(int x) const { return wt[x]; }
  __device__ __forceinline__ cplx<R> xp(int x) const { return wt[w + x]; }
  __device__ __forceinline__ cplx<R> ym(int y) const { return wt[2 * w + y]; }
  __device__ __forceinline__ cplx<R> yp(int y) const { return wt[2 * w + h + y]; }
};

template <typename R>
__device__ __forceinline__ Region<R> make_region(int ox, int oy, int w, int h, cplx<R> *wts) {
  Region<R> g;
  g.wt = wts;
  g.ox = ox;
  g.oy = oy;
  g.w = w;
  g.h = h;
  g.invw = 1.0f / (float)w;
  g.invh2 = 1.0f / (float)((w + 1) >> 1);
  return g;
}

__device__ __forceinline__ bool interior(const int i, const int j, const int n0, const int n1) {
  return i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2;
}

// The level's 1D weights over region A's columns and rows (0 off the
// interior, where they are never used), w + h <= NP, one entry per thread:
// read into registers first, written to LDS once the other staging loads of
// the block have been issued.
template <typename R>
struct WeightRead {
  cplx<R> m, p;
  bool in;
};

template <typename R>
__device__ __forceinline__ WeightRead<R> read_weights(const Grid<R> &g, const Region<R> &A) {
  const int q = threadIdx.x;
  const bool col = q < A.w;
  const int v = col ? A.ox + q : A.oy + q - A.w;
  const int n = col ? g.n0 : g.n1;
  const bool in = q < A.w + A.h && v >= 1 && v <= n - 2;
  const int vc = in ? v : 1;
  WeightRead<R> w;
  w.m = col ? g.cm0[vc] : g.cm1[vc];
  w.p = col ? g.cp0[vc] : g.cp1[vc];
  w.in = in;  // applied at the write, so no use follows the loads here
  return w;
}

template <typename R>
__device__ __forceinline__ void write_weights(const Region<R> &A, const WeightRead<R> &w) {
  const int q = threadIdx.x;
  const cplx<R> m = w.in ? w.m : zc<R>(), p = w.in ? w.p : zc<R>();
  if (q < A.w) {
    A.wt[q] = m;
    A.wt[A.w + q] = p;
  } else if (q < A.w + A.h) {
    A.wt[A.w + q] = m;              // ym at 2w + (q - w)
    A.wt[A.w + A.h + q] = p;        // yp at 2w + h + (q - w)
  }
}

// Stages one level over a region of WH nodes into LDS: t and b (when wanted)
// and the inverse diagonal of every node, 0 off the interior.  The loop runs
// a fixed number of slots per thread with clamped, unconditional loads, so
// all loads of the block are in flight before the first is used.
template <typename R, int WH, bool T, bool B>
__device__ __forceinline__ void stage_level(const Grid<R> &g, const Region<R> &A, const cplx<R> *t, const cplx<R> *b,
                                            cplx<R> *at, cplx<R> *ab, cplx<R> *ad) {
  constexpr int S = (WH + NP - 1) / NP;
  cplx<R> tv[S], bv[S], wx[S], wy[S];
  R kv[S];
  bool in[S];
#pragma unroll
  for (int s = 0; s < S; s++) {
    const int q = threadIdx.x + s * NP;
    int x, y;
    xy_of(q, A.w, A.invw, x, y);
    const int i = A.ox + x, j = A.oy + y;
    in[s] = q < WH && interior(i, j, g.n0, g.n1);
    const int ic = in[s] ? i : 1, jc = in[s] ? j : 1;
    const int64_t p = (int64_t)jc * g.n0 + ic;
    if (T) tv[s] = t[p];
    if (B) bv[s] = b[p];
    kv[s] = g.k2[p];
    wx[s] = g.cm0[ic] + g.cp0[ic];
    wy[s] = g.cm1[jc] + g.cp1[jc];
  }
#pragma unroll
  for (int s = 0; s < S; s++) {
    const int q = threadIdx.x + s * NP;
    if (q < WH) {
      if (T) at[q] = in[s] ? tv[s] : zc<R>();
      if (B) ab[q] = in[s] ? bv[s] : zc<R>();
      ad[q] = in[s] ? inv_p(wx[s] + wy[s] + (kv[s] * g.beta + g.c)) : zc<R>();
    }
  }
}

// ---------------------------------------------------------------- down
// Zero-guess red-black sweep and residual of one level over region A
// (b, d given in LDS; t, r written to LDS), the relaxed iterate written to
// global memory on the owned sub-rectangle [o0, o1) x [p0, p1) (relative).
// Ends without a barrier.
template <typename R>
__device__ void down_sweep(const Grid<R> &g, const Region<R> &A, const cplx<R> *ab, const cplx<R> *ad, cplx<R> *at,
                           cplx<R> *ar, R omega, cplx<R> *t_out, int o0, int o1, int p0, int p1) {
  const int tid = threadIdx.x, n0 = g.n0, n1 = g.n1, W = A.w;
  const R om1 = R(1) - omega;
  const int H2 = (W + 1) >> 1, np = A.h * H2;
  // red from zero: omega b / D; black 0
  for (int q = tid; q < A.w * A.h; q += NP) {
    int x, y;
    xy_of(q, W, A.invw, x, y);
    const int i = A.ox + x, j = A.oy + y;
    at[q] = (((i + j) & 1) == 0) ? omega * (ab[q] * ad[q]) : zc<R>();
  }
  __syncthreads();
  // black relaxation and the black residual (1 - w)(b + o)
  for (int q = tid; q < np; q += NP) {
    int h, y;
    xy_of(q, H2, A.invh2, h, y);
    const int j = A.oy + y;
    const int x = 2 * h + ((A.ox + 2 * h + j + 1) & 1);  // the pair's black node
    const int i = A.ox + x;
    if (x >= 1 && x <= W - 2 && y >= 1 && y <= A.h - 2 && interior(i, j, n0, n1)) {
      const int p = y * W + x;
      const cplx<R> tb = ab[p] + (A.xm(x) * at[p - 1] + A.xp(x) * at[p + 1] + A.ym(y) * at[p - W] +
                                  A.yp(y) * at[p + W]);
      at[p] = omega * (tb * ad[p]);
      ar[p] = om1 * tb;
    }
  }
  __syncthreads();
  // red residual (1 - w) b + o; the relaxed iterate of the owned nodes out
  for (int q = tid; q < np; q += NP) {
    int h, y;
    xy_of(q, H2, A.invh2, h, y);
    const int j = A.oy + y;
    const int x = 2 * h + ((A.ox + 2 * h + j) & 1);  // the pair's red node
    const int i = A.ox + x;
    if (x >= 1 && x <= W - 2 && y >= 1 && y <= A.h - 2 && interior(i, j, n0, n1)) {
      const int p = y * W + x;
      ar[p] = om1 * ab[p] + (A.xm(x) * at[p - 1] + A.xp(x) * at[p + 1] + A.ym(y) * at[p - W] +
                             A.yp(y) * at[p + W]);
    }
    if (y >= p0 && y < p1 && j < n1) {
      const int xa = 2 * h;
      for (int e = 0; e < 2; e++) {
        const int xx = xa + e, ii = A.ox + xx;
        if (xx >= o0 && xx < o1 && ii < n0) t_out[(int64_t)j * n0 + ii] = at[y * W + xx];
      }
    }
  }
}

// full weighting of the residual ar (region A of the fine level) onto the
// coarse nodes (cx0 + X, cy0 + Y), 0 <= X < cw, 0 <= Y < ch; A's origin is
// (2 cx0 - 3, 2 cy0 - 3).  f(q, value) receives each coarse value (0 off the
// coarse interior).
template <typename R, typename F>
__device__ __forceinline__ void restrict_fw(const Grid<R> &c, const Region<R> &A, const cplx<R> *ar, int cx0, int cy0,
                                            int cw, int ch, F &&f) {
  const float invcw = 1.0f / (float)cw;
  const int W = A.w;
  for (int q = threadIdx.x; q < cw * ch; q += NP) {
    int X, Y;
    xy_of(q, cw, invcw, X, Y);
    const int I = cx0 + X, J = cy0 + Y;
    cplx<R> acc = zc<R>();
    if (interior(I, J, c.n0, c.n1)) {
      const cplx<R> *r0 = ar + (2 * Y + 3) * W + 2 * X + 3;
      acc = R(0.25) * r0[0] + R(0.125) * (r0[-1] + r0[1] + r0[-W] + r0[W]) +
            R(0.0625) * (r0[-W - 1] + r0[-W + 1] + r0[W - 1] + r0[W + 1]);
    }
    f(q, X, Y, I, J, acc);
  }
}

// Block tile: C x CY nodes of level l + 2 at (I0, J0).  Mid region (level
// l+1): origin (2 I0 - 3, 2 J0 - 3), (2C + 5) x (2CY + 5); fine region
// (level l): origin twice that minus 3, (4C + 15) x (4CY + 15).
template <typename R, int C, int CY, bool MR>
__global__ __launch_bounds__(NP) void k_down2_rb(Grid<R> f, Grid<R> m, Grid<R> c, const cplx<R> *__restrict__ b,
                                                 cplx<R> *__restrict__ t_f, cplx<R> *__restrict__ b_m,
                                                 cplx<R> *__restrict__ t_m, cplx<R> *__restrict__ rc, R omega,
                                                 int tiles_x, int tiles, RhsSet rs) {
  constexpr int MW = 2 * C + 5, MH = 2 * CY + 5;
  constexpr int AW = 2 * MW + 5, AH = 2 * MH + 5;
  __shared__ cplx<R> Ab[AW * AH], Ad[AW * AH], At[AW * AH], Ar[AW * AH];
  __shared__ cplx<R> Mb[MW * MH], Md[MW * MH], Mt[MW * MH], Mr[MW * MH];
  __shared__ cplx<R> Aw[2 * (AW + AH)], Mw[2 * (MW + MH)];
  const int tile = xcd_tile(tiles);
  if (tile < 0) return;
  if constexpr (MR) {
    const int64_t q = rhs_index(rs);
    const int64_t sf = rhs_stride((int64_t)f.n0 * f.n1), sm = rhs_stride((int64_t)m.n0 * m.n1);
    b += q * sf;
    t_f += q * sf;
    b_m += q * sm;
    t_m += q * sm;
    rc += q * rhs_stride((int64_t)c.n0 * c.n1);
  }
  const int I0 = (tile % tiles_x) * C, J0 = (tile / tiles_x) * CY;
  const Region<R> M = make_region(2 * I0 - 3, 2 * J0 - 3, MW, MH, Mw);
  const Region<R> A = make_region(2 * M.ox - 3, 2 * M.oy - 3, AW, AH, Aw);
  static_assert(AW + AH <= NP && MW + MH <= NP, "weights are staged one entry per thread");
  // one memory round trip: the weights of both levels, b and the inverse
  // diagonal of the fine region, the inverse diagonal of the mid region (fixed
  // trip counts and clamped, unconditional loads: every load is issued before
  // the first use)
  const WeightRead<R> wa = read_weights(f, A), wm = read_weights(m, M);
  stage_level<R, AW * AH, false, true>(f, A, nullptr, b, nullptr, Ab, Ad);
  stage_level<R, MW * MH, false, false>(m, M, nullptr, nullptr, nullptr, nullptr, Md);
  write_weights(A, wa);
  write_weights(M, wm);
  __syncthreads();
  // level l; owned fine nodes [4 I0, 4 I0 + 4C) -> relative [9, 9 + 4C)
  down_sweep(f, A, Ab, Ad, At, Ar, omega, t_f, 9, 9 + 4 * C, 9, 9 + 4 * CY);
  __syncthreads();
  // b_{l+1} over the mid region; owned mid nodes [2 I0, 2 I0 + 2C) -> [3, 3 + 2C)
  restrict_fw(m, A, Ar, M.ox, M.oy, MW, MH, [&](int q, int X, int Y, int I, int J, cplx<R> v) {
    Mb[q] = v;
    if (X >= 3 && X < 3 + 2 * C && Y >= 3 && Y < 3 + 2 * CY && I < m.n0 && J < m.n1)
      b_m[(int64_t)J * m.n0 + I] = v;
  });
  __syncthreads();
  // level l + 1
  down_sweep(m, M, Mb, Md, Mt, Mr, omega, t_m, 3, 3 + 2 * C, 3, 3 + 2 * CY);
  __syncthreads();
  // b_{l+2} on the tile
  restrict_fw(c, M, Mr, I0, J0, C, CY, [&](int q, int X, int Y, int I, int J, cplx<R> v) {
    if (I < c.n0 && J < c.n1) rc[(int64_t)J * c.n0 + I] = v;
  });
}

// ------------------------------------------------------------------ up
// v = t + P e over region A (e: the coarse values in LDS over region E, A's
// nodes interpolate from E's), then the red sweep on A minus its outer ring,
// then the black sweep on the sub-rectangle [o0, o1) x [p0, p1) (relative),
// whose final values (both colours) are handed to out(q, x, y, i, j, value).
template <typename R, typename F>
__device__ void up_sweep(const Grid<R> &g, const Region<R> &A, const cplx<R> *ab, const cplx<R> *ad,
                         const cplx<R> *at, cplx<R> *av, const Region<R> &E, const cplx<R> *ev, R omega, int o0, int o1,
                         int p0, int p1, F &&out) {
  const int tid = threadIdx.x, n0 = g.n0, n1 = g.n1, W = A.w, EW = E.w;
  const R om1 = R(1) - omega;
  const int H2 = (W + 1) >> 1, np = A.h * H2;
  for (int q = tid; q < A.w * A.h; q += NP) {
    int x, y;
    xy_of(q, W, A.invw, x, y);
    const int i = A.ox + x, j = A.oy + y;
    cplx<R> v = zc<R>();
    if (interior(i, j, n0, n1)) {
      const cplx<R> *e0 = ev + ((j >> 1) - E.oy) * EW + ((i >> 1) - E.ox);
      const cplx<R> e1 = (i & 1) ? e0[1] : zc<R>();
      const cplx<R> e2 = (j & 1) ? e0[EW] : zc<R>();
      const cplx<R> e3 = ((i & 1) && (j & 1)) ? e0[EW + 1] : zc<R>();
      const R wx = (i & 1) ? R(0.5) : R(1), wy = (j & 1) ? R(0.5) : R(1);
      v = at[q] + (wx * wy) * (e0[0] + e1 + e2 + e3);
    }
    av[q] = v;
  }
  __syncthreads();
  for (int colour = 0; colour < 2; colour++) {
    for (int q = tid; q < np; q += NP) {
      int h, y;
      xy_of(q, H2, A.invh2, h, y);
      const int j = A.oy + y;
      const int x = 2 * h + ((A.ox + 2 * h + j + colour) & 1);  // the pair's node of this colour
      const int i = A.ox + x;
      const bool ring_ok = colour == 0 ? (x >= 1 && x <= W - 2 && y >= 1 && y <= A.h - 2)
                                       : (x >= o0 && x < o1 && y >= p0 && y < p1);
      if (ring_ok && interior(i, j, n0, n1)) {
        const int p = y * W + x;
        const cplx<R> o = A.xm(x) * av[p - 1] + A.xp(x) * av[p + 1] + A.ym(y) * av[p - W] + A.yp(y) * av[p + W];
        av[p] = om1 * av[p] + omega * ((ab[p] + o) * ad[p]);
      }
    }
    __syncthreads();
  }
  for (int q = tid; q < A.w * A.h; q += NP) {
    int x, y;
    xy_of(q, W, A.invw, x, y);
    if (x >= o0 && x < o1 && y >= p0 && y < p1) out(q, x, y, A.ox + x, A.oy + y, av[q]);
  }
}

// load t, b and the inverse diagonal of region A of level g (0 off the
// interior)
// Block tile: TX x TY nodes of level l at (x0, y0), x0 and y0 even.  Fine
// region: (x0 - 2, y0 - 2), (TX + 4) x (TY + 4).  Its nodes interpolate from
// mid nodes E = (x0/2 - 1, y0/2 - 1), (TX/2 + 3) x (TY/2 + 3), whose final
// values need the mid sweep over E plus a 2-node halo (region F), whose nodes
// interpolate from coarse region G.
template <typename R, int TX, int TY, bool MR>
__global__ __launch_bounds__(NP) void k_up2_rb(Grid<R> f, Grid<R> m, Grid<R> c, const cplx<R> *__restrict__ b_f,
                                               const cplx<R> *__restrict__ t_f, const cplx<R> *__restrict__ b_m,
                                               const cplx<R> *__restrict__ t_m, const cplx<R> *__restrict__ ec,
                                               cplx<R> *__restrict__ u_out, R omega, int tiles_x, int tiles,
                                               RhsSet rs) {
  constexpr int AW = TX + 4, AH = TY + 4;
  constexpr int EW = TX / 2 + 3, EH = TY / 2 + 3;
  constexpr int FW = EW + 4, FH = EH + 4;
  constexpr int GW = FW / 2 + 3, GH = FH / 2 + 3;
  __shared__ cplx<R> At[AW * AH], Ab[AW * AH], Ad[AW * AH], Av[AW * AH];
  __shared__ cplx<R> Ft[FW * FH], Fb[FW * FH], Fd[FW * FH], Fv[FW * FH];
  __shared__ cplx<R> Ge[GW * GH];
  __shared__ cplx<R> Aw[2 * (AW + AH)], Fw[2 * (FW + FH)];
  const int tile = xcd_tile(tiles);
  if (tile < 0) return;
  if constexpr (MR) {
    const int64_t q = rhs_index(rs);
    const int64_t sf = rhs_stride((int64_t)f.n0 * f.n1), sm = rhs_stride((int64_t)m.n0 * m.n1);
    b_f += q * sf;
    t_f += q * sf;
    u_out += q * sf;
    b_m += q * sm;
    t_m += q * sm;
    ec += q * rhs_stride((int64_t)c.n0 * c.n1);
  }
  const int tid = threadIdx.x;
  const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
  const Region<R> A = make_region(x0 - 2, y0 - 2, AW, AH, Aw);
  // mid nodes the fine region interpolates from: E = (x0/2 - 1, y0/2 - 1),
  // EW x EH; their sweep needs F = E plus a 2-node halo
  const Region<R> F = make_region(x0 / 2 - 3, y0 / 2 - 3, FW, FH, Fw);
  // coarse nodes under F: from floor(F.ox / 2) (F.ox may be odd or negative)
  const Region<R> G = make_region(F.ox >> 1, F.oy >> 1, GW, GH, (cplx<R> *)nullptr);
  static_assert(AW + AH <= NP && FW + FH <= NP && GW * GH <= NP, "staged one entry per thread");
  // one memory round trip: the weights of both levels, the coarse correction
  // over G, t, b and the inverse diagonals of both levels (clamped,
  // unconditional loads, all issued before the first use)
  const WeightRead<R> wa = read_weights(f, A), wf = read_weights(m, F);
  cplx<R> ge;
  bool ge_in;
  {
    int x, y;
    xy_of(tid, GW, G.invw, x, y);
    const int I = G.ox + x, J = G.oy + y;
    const bool in = tid < GW * GH && I >= 0 && I < c.n0 && J >= 0 && J < c.n1;
    ge_in = in;
    ge = ec[in ? (int64_t)J * c.n0 + I : 0];
  }
  stage_level<R, FW * FH, true, true>(m, F, t_m, b_m, Ft, Fb, Fd);
  stage_level<R, AW * AH, true, true>(f, A, t_f, b_f, At, Ab, Ad);
  write_weights(A, wa);
  write_weights(F, wf);
  if (tid < GW * GH) Ge[tid] = ge_in ? ge : zc<R>();
  __syncthreads();
  // level l + 1 over F; its final values on E (relative [2, 2 + EW)) into Ge's
  // successor: stored in Fv itself (the up sweep leaves them there)
  up_sweep(m, F, Fb, Fd, Ft, Fv, G, Ge, omega, 2, 2 + EW, 2, 2 + EH,
           [&](int, int, int, int, int, cplx<R>) {});
  __syncthreads();
  // level l over A, interpolating from the mid values: E lies inside F at
  // offset 2, so the mid values are read from Fv with F's geometry
  up_sweep(f, A, Ab, Ad, At, Av, F, Fv, omega, 2, 2 + TX, 2, 2 + TY,
           [&](int q, int x, int y, int i, int j, cplx<R> v) {
             if (i < f.n0 && j < f.n1) u_out[(int64_t)j * f.n0 + i] = v;
           });
}

}  // namespace

template <typename R>
void launch_down2_rb(const Grid<R> &f, const Grid<R> &m, const Grid<R> &c, const cplx<R> *b, cplx<R> *t_f,
                     cplx<R> *b_m, cplx<R> *t_m, cplx<R> *rc, R omega, hipStream_t s, const RhsSet &rs) {
  constexpr int C = 8, CY = sizeof(R) == 4 ? 4 : 2;
  const int tx = (c.n0 + C - 1) / C;
  const int tiles = tx * ((c.n1 + CY - 1) / CY);
  if (multi_rhs(rs))
    launch_k((k_down2_rb<R, C, CY, true>), dim3(xcd_padded(tiles), rs.count), dim3(NP), 0, s, f, m, c, b, t_f, b_m,
             t_m, rc, omega, tx, tiles, rs);
  else
    launch_k((k_down2_rb<R, C, CY, false>), dim3(xcd_padded(tiles)), dim3(NP), 0, s, f, m, c, b, t_f, b_m, t_m, rc,
             omega, tx, tiles, rs);
}

template <typename R>
void launch_up2_rb(const Grid<R> &f, const Grid<R> &m, const Grid<R> &c, const cplx<R> *b_f, const cplx<R> *t_f,
                   const cplx<R> *b_m, const cplx<R> *t_m, const cplx<R> *ec, cplx<R> *u_out, R omega,
                   hipStream_t s, const RhsSet &rs) {
  constexpr int TX = 32, TY = sizeof(R) == 4 ? 16 : 8;
  const int tx = (f.n0 + TX - 1) / TX;
  const int tiles = tx * ((f.n1 + TY - 1) / TY);
  if (multi_rhs(rs))
    launch_k((k_up2_rb<R, TX, TY, true>), dim3(xcd_padded(tiles), rs.count), dim3(NP), 0, s, f, m, c, b_f, t_f, b_m,
             t_m, ec, u_out, omega, tx, tiles, rs);
  else
    launch_k((k_up2_rb<R, TX, TY, false>), dim3(xcd_padded(tiles)), dim3(NP), 0, s, f, m, c, b_f, t_f, b_m, t_m, ec,
             u_out, omega, tx, tiles, rs);
}

template void launch_down2_rb<double>(const Grid<double> &, const Grid<double> &, const Grid<double> &,
                                      const cplx<double> *, cplx<double> *, cplx<double> *, cplx<double> *,
                                      cplx<double> *, double, hipStream_t, const RhsSet &);
template void launch_down2_rb<float>(const Grid<float> &, const Grid<float> &, const Grid<float> &,
                                     const cplx<float> *, cplx<float> *, cplx<float> *, cplx<float> *,
                                     cplx<float> *, float, hipStream_t, const RhsSet &);
template void launch_up2_rb<double>(const Grid<double> &, const Grid<double> &, const Grid<double> &,
                                    const cplx<double> *, const cplx<double> *, const cplx<double> *,
                                    const cplx<double> *, const cplx<double> *, cplx<double> *, double,
                                    hipStream_t, const RhsSet &);
template void launch_up2_rb<float>(const Grid<float> &, const Grid<float> &, const Grid<float> &,
                                   const cplx<float> *, const cplx<float> *, const cplx<float> *,
                                   const cplx<float> *, const cplx<float> *, cplx<float> *, float, hipStream_t,
                                   const RhsSet &);

}  // namespace ecs
