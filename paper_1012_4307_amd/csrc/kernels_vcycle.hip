// kernels_vcycle.hip -- fused 2D kernels of the V(1,1) red-black cycle (the
// QD set-up of bin Zubair, Reps, Vanroose, Sec. 4.2: one red-black SOR sweep
// before and after the coarse-grid correction, full weighting, bilinear
// interpolation).  Each level is visited by exactly two kernels:
//
//   down: u = S_rb(0; b) (zero-guess sweep), rc = FW(b - M u)
//         reads b, k^2 once, writes the coarse residual (u is not stored)
//   up:   u = S_rb(0; b) again, v = u + P ec, u_out = S_rb(v; b) (post-sweep,
//         out of place); reads ec, b, k^2 once, writes u_out
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
#include "ecs_krylov.h"

namespace ecs {

namespace {

constexpr int NT = 256;

template <typename R>
__device__ __forceinline__ cplx<R> zero_c() {
  return mk<R>(0, 0);
}

// Both kernels first issue every global load of the block (register arrays
// of RPW rows per thread, unrolled, so all are in flight together).  A thread
// keeps the values of its own nodes (b, the inverse diagonal, its iterate) in
// registers across the phases; only the iterate and the residual, which
// neighbours read, go through LDS.
//
// Pair layout: lane l owns the two adjacent columns 2l, 2l + 1 of the staged
// region.  In every row one of them is red and the other black, so each lane
// has exactly one node of each colour per row, and a colour phase keeps every
// lane busy (with one lane per column, half the lanes of every instruction of
// a colour phase would idle).  The 4 waves of a block take every fourth row,
// so all rows of a wave have one parity and the colour of column 2l is the
// same for the whole wave.  LDS holds the red and the black values of each
// row apart, [row][pair]: a node's four neighbours are the other colour of
// its own pair, of the pair to one side, and of its own pair one row up and
// down.
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

// inverse diagonal inside the fused cycle: in FP32 the hardware reciprocal
// (1 ulp) replaces the correctly rounded division
template <typename R>
__device__ __forceinline__ cplx<R> inv_cycle(cplx<R> d) {
  R s;
  if constexpr (sizeof(R) == 4) s = __builtin_amdgcn_rcpf(abs2(d));
  else s = R(1) / abs2(d);
  return mk<R>(d.re * s, -d.im * s);
}

template <typename R>
__device__ __forceinline__ cplx<R> sel(bool c, cplx<R> a, cplx<R> b) {
  return c ? a : b;
}

// ----------------------------------------------------------------- down
// Block tile: CX = 61 coarse columns x CY coarse rows from (I0, J0); owned
// fine nodes [2 I0, 2 I0 + 122) x [2 J0, 2 J0 + 2 CY).  Staged fine region:
// columns 2 I0 - 3 + [0, 127) (the second column of pair 63 idles), rows
// 2 J0 - 3 + [0, 2 CY + 5): halo 3 below, 2 above, because the FW stencil of
// the tile's coarse nodes reads residuals one node out, a residual reads the
// relaxed iterate one further out, and a relaxed black node reads red values
// one further still.
//
// SRC selects the right-hand side: kDownSrcB reads b; kDownSrcP and kDownSrcS
// stage the Bi-CGSTAB vectors it is formed from instead (r, p, v or r, v),
// form it per staged node and store it at the owned nodes (boundary nodes,
// read as 0, get 0).
template <typename R, int CY, int SRC, bool MR>
__global__ __launch_bounds__(NT) void k_down_rb(Grid<R> f, Grid<R> c, const cplx<R> *__restrict__ b,
                                                const DownSrc<R> src, cplx<R> *__restrict__ rc, R omega,
                                                int tiles_x, int tiles, RhsSet rs) {
  constexpr int CX = 61;
  constexpr int WX = 2 * CX + 5;          // 127 staged columns
  constexpr int WY = 2 * CY + 5;
  constexpr int RPW = (WY + 3) / 4;       // rows per wave
  // relaxed iterate by colour; the residual by colour, the red one in the
  // red iterate's slots (in the residual phase a lane reads only its own red
  // node there, before overwriting it): three arrays keep eight blocks per CU
  __shared__ cplx<R> sR[WY][64], sB[WY][64], rB[WY][64];
  cplx<R>(*const rR)[64] = sR;
  // the wave index is uniform: row indices and row weights live in scalars
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = xcd_tile(tiles);
  if (tile < 0) return;
  if constexpr (MR) {
    // this block's right-hand side (a separate instantiation: the slot is a
    // load the single right-hand side path does not wait for)
    const int64_t q = rhs_index(rs);
    b += q * rhs_stride((int64_t)f.n0 * f.n1);
    rc += q * rhs_stride((int64_t)c.n0 * c.n1);
  }
  const int I0 = (tile % tiles_x) * CX, J0 = (tile / tiles_x) * CY;
  const int gx0 = 2 * I0 - 3, gy0 = 2 * J0 - 3;
  const int n0 = f.n0, n1 = f.n1;
  const R om1 = R(1) - omega;
  // the lane's columns a = 2 lane, b = 2 lane + 1 (relative)
  const int ia = gx0 + 2 * lane, ib = ia + 1;
  const bool ina = 2 * lane < WX && ia >= 1 && ia <= n0 - 2;
  const bool inb = 2 * lane + 1 < WX && ib >= 1 && ib <= n0 - 2;
  // column a is red in this wave's rows iff ia + j is even (one parity for all)
  const bool ared = ((ia + gy0 + wv) & 1) == 0;
  const bool inR = ared ? ina : inb, inBk = ared ? inb : ina;
  const int iR = ared ? ia : ib, iBk = ared ? ib : ia;
  const cplx<R> xmR = inR ? f.cm0[iR] : zero_c<R>(), xpR = inR ? f.cp0[iR] : zero_c<R>();
  const cplx<R> xmB = inBk ? f.cm0[iBk] : zero_c<R>(), xpB = inBk ? f.cp0[iBk] : zero_c<R>();
  // interior rows of the staged window through buffer resources: halo and
  // boundary nodes read as 0
  const int jl = min(max(gy0, 1), n1 - 1), jh = min(max(gy0 + WY, 1), n1 - 1);
  const __amdgpu_buffer_rsrc_t rb = rows_rsrc(b, jl, jh, n0), rk = rows_rsrc(f.k2, jl, jh, n0);
  const uint32_t obR = col_off<cplx<R>>(inR, iR), obB = col_off<cplx<R>>(inBk, iBk);
  const uint32_t okR = col_off<R>(inR, iR), okB = col_off<R>(inBk, iBk);

  cplx<R> bR[RPW], bB[RPW], dR[RPW], dB[RPW], cym[RPW], cyp[RPW];
  R kR[RPW], kB[RPW];
  // the vectors the right-hand side is formed from (SRC != kDownSrcB)
  const __amdgpu_buffer_rsrc_t rr = rows_rsrc(src.r, jl, jh, n0), rv = rows_rsrc(src.v, jl, jh, n0),
                               rp = rows_rsrc(SRC == kDownSrcP ? src.p : src.r, jl, jh, n0);
  cplx<R> xR[RPW], xB[RPW], vR[RPW], vB[RPW], pR[RPW], pB[RPW];
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    const int j = gy0 + ly;
    const bool yin = ly < WY && j >= 1 && j <= n1 - 2;
    const int jc = yin ? j : 1;
    cym[r] = yin ? f.cm1[jc] : zero_c<R>();
    cyp[r] = yin ? f.cp1[jc] : zero_c<R>();
    const uint32_t qb = row_off<cplx<R>>(j - jl, n0), qk = row_off<R>(j - jl, n0);
    if constexpr (SRC == kDownSrcB) {
      bR[r] = ld_c(rb, obR + qb, cplx<R>());
      bB[r] = ld_c(rb, obB + qb, cplx<R>());
    } else {
      xR[r] = ld_c(rr, obR + qb, cplx<R>());
      xB[r] = ld_c(rr, obB + qb, cplx<R>());
      vR[r] = ld_c(rv, obR + qb, cplx<R>());
      vB[r] = ld_c(rv, obB + qb, cplx<R>());
      if constexpr (SRC == kDownSrcP) {
        pR[r] = ld_c(rp, obR + qb, cplx<R>());
        pB[r] = ld_c(rp, obB + qb, cplx<R>());
      }
    }
    kR[r] = ld_r(rk, okR + qk, R());
    kB[r] = ld_r(rk, okB + qk, R());
  }
  if constexpr (SRC != kDownSrcB) {
    // the same expressions as the separate update kernels
    if constexpr (SRC == kDownSrcP) {
      const cplx<R> beta = cvt<R>(src.S->beta), om_s = cvt<R>(src.S->omega);
#pragma unroll
      for (int r = 0; r < RPW; r++) {
        bR[r] = xR[r] + beta * (pR[r] - om_s * vR[r]);
        bB[r] = xB[r] + beta * (pB[r] - om_s * vB[r]);
      }
    } else {
      const cplx<R> alpha = cvt<R>(src.S->alpha);
#pragma unroll
      for (int r = 0; r < RPW; r++) {
        bR[r] = xR[r] - alpha * vR[r];
        bB[r] = xB[r] - alpha * vB[r];
      }
    }
    // owned nodes: staged columns [3, 3 + 2 CX), rows [3, 3 + 2 CY)
    const int ca = 2 * lane;
    const bool owna = ca >= 3 && ca < 3 + 2 * CX && ia < n0;
    const bool ownb = ca + 1 >= 3 && ca + 1 < 3 + 2 * CX && ib < n0;
#pragma unroll
    for (int r = 0; r < RPW; r++) {
      const int ly = wv + 4 * r, j = gy0 + ly;
      if (ly >= 3 && ly < 3 + 2 * CY && j < n1) {
        cplx<R> *row = src.out + (int64_t)j * n0;
        // component selects: a select of the structs goes through scratch
        // memory in FP64
        const cplx<R> va = mk<R>(ared ? bR[r].re : bB[r].re, ared ? bR[r].im : bB[r].im);
        const cplx<R> vb = mk<R>(ared ? bB[r].re : bR[r].re, ared ? bB[r].im : bR[r].im);
        if (owna) row[ia] = va;
        if (ownb) row[ib] = vb;
      }
    }
  }
  // inverse diagonals; red relaxation from zero: omega b / D.  Row
  // conditions depend on the wave (uniform) and are tested apart from the
  // lane conditions, so the compiler branches on them instead of carrying a
  // per-lane exit state through the unrolled row loops.
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    if (ly < WY) {
      const int j = gy0 + ly;
      const bool yin = j >= 1 && j <= n1 - 2;
      dR[r] = (yin && inR) ? inv_cycle(xmR + xpR + cym[r] + cyp[r] + (kR[r] * f.beta + f.c)) : zero_c<R>();
      dB[r] = (yin && inBk) ? inv_cycle(xmB + xpB + cym[r] + cyp[r] + (kB[r] * f.beta + f.c)) : zero_c<R>();
      sR[ly][lane] = omega * (bR[r] * dR[r]);
      sB[ly][lane] = zero_c<R>();
    }
  }
  __syncthreads();
  // black relaxation and the black residual (1 - w)(b + o).  The black node's
  // red neighbours: its own pair's red and the red of pair lane + 1 (black in
  // column a... mirrored: lane - 1) in its row, its own pair's red one row up
  // and down.
  const int side = ared ? 1 : -1;  // pair holding the black node's other row neighbour
  const bool pin = lane + side >= 0 && lane + side < 64;
  const int ps = pin ? lane + side : lane;
  // black in column b: left = own red, right = red of lane + 1; in column a:
  // left = red of lane - 1, right = own red.  Weights of the own-pair and the
  // other-pair neighbour:
  const cplx<R> wBo = ared ? xmB : xpB, wBn = ared ? xpB : xmB;
  cplx<R> resB[RPW], tB[RPW];
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    resB[r] = tB[r] = zero_c<R>();
    if (ly >= 1 && ly <= WY - 2) {
      if (pin) {
        const cplx<R> tb =
            bB[r] + (wBo * sR[ly][lane] + wBn * sR[ly][ps] + cym[r] * sR[ly - 1][lane] + cyp[r] * sR[ly + 1][lane]);
        tB[r] = omega * (tb * dB[r]);
        resB[r] = om1 * tb;
        sB[ly][lane] = tB[r];
      }
    }
  }
  __syncthreads();
  // red residual (1 - w) b + o from the relaxed black neighbours: own black
  // and the black of pair lane - side (red in column a: left = black of
  // lane - 1, right = own black); zero off the interior.  Residuals to LDS.
  // The relaxed iterate itself is not stored: the up kernel recomputes it.
  const int qs = lane - side;
  const bool qin = qs >= 0 && qs < 64;
  const int pq = qin ? qs : lane;
  const cplx<R> wRo = ared ? xpR : xmR, wRn = ared ? xmR : xpR;
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    if (ly < WY) {
      const int j = gy0 + ly;
      const bool yin = j >= 1 && j <= n1 - 2;
      cplx<R> resR = zero_c<R>();
      if (yin && ly >= 1 && ly <= WY - 2) {
        if (inR && qin)
          resR = om1 * bR[r] +
                 (wRo * sB[ly][lane] + wRn * sB[ly][pq] + cym[r] * sB[ly - 1][lane] + cyp[r] * sB[ly + 1][lane]);
      }
      rR[ly][lane] = resR;
      rB[ly][lane] = (yin && inBk) ? resB[r] : zero_c<R>();
    }
  }
  __syncthreads();
  // full weighting onto the owned coarse nodes: lane = coarse column.  The
  // coarse node (I, J) sits on the red fine node in column b of pair P =
  // I - I0 + 1, row y = 2 (J - J0) + 3 (rows y +- 1 have the other colouring).
  if (lane < CX) {
    const int I = I0 + lane, P = lane + 1;
    for (int cy = wv; cy < CY; cy += 4) {
      const int J = J0 + cy;
      if (I >= c.n0 || J >= c.n1) continue;
      cplx<R> acc = zero_c<R>();
      if (I >= 1 && I <= c.n0 - 2 && J >= 1 && J <= c.n1 - 2) {
        const int y = 3 + 2 * cy;
        acc = R(0.25) * rR[y][P] + R(0.125) * (rB[y][P] + rB[y][P + 1] + rB[y - 1][P] + rB[y + 1][P]) +
              R(0.0625) * (rR[y - 1][P] + rR[y - 1][P + 1] + rR[y + 1][P] + rR[y + 1][P + 1]);
      }
      rc[(int64_t)J * c.n0 + I] = acc;
    }
  }
}

// ------------------------------------------------------------------- up
// Block tile: TX = 120 x TY fine nodes at (x0, y0), both even.  The
// pre-smoothed iterate t of the down pass is not stored: it is recomputed
// here from b (the zero-guess red relaxation, then the black one), which
// costs one phase and a wider halo but saves writing and re-reading a fine
// vector.  Staged fine region: columns x0 - 4 + [0, 128) (pairs 2..61 owned),
// rows y0 - 3 + [0, TY + 6): red t on ring 3 feeds black t on ring 2, the red
// relaxation on ring 1 reads black values on ring 2, and the black relaxation
// on the tile reads red values on ring 1.  Column a = x0 - 4 + 2 lane is even,
// so both columns of pair l interpolate from coarse column x0/2 - 2 + l
// (= staged coarse column l).
template <typename R, int TY, bool MR>
__global__ __launch_bounds__(NT) void k_up_rb(Grid<R> f, Grid<R> c, const cplx<R> *__restrict__ b,
                                              const cplx<R> *__restrict__ ec, cplx<R> *__restrict__ u_out, R omega,
                                              int tiles_x, int tiles, RhsSet rs) {
  constexpr int TX = 120;
  constexpr int WY = TY + 6;
  constexpr int RPW = (WY + 3) / 4;
  constexpr int CWX = TX / 2 + 5, CWY = TY / 2 + 3;
  __shared__ cplx<R> sR[WY][64], sB[WY][64];
  __shared__ cplx<R> se[CWY][CWX];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = xcd_tile(tiles);
  if (tile < 0) return;
  if constexpr (MR) {
    const int64_t q = rhs_index(rs), sf = rhs_stride((int64_t)f.n0 * f.n1);
    b += q * sf;
    u_out += q * sf;
    ec += q * rhs_stride((int64_t)c.n0 * c.n1);
  }
  const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
  const int gx0 = x0 - 4, gy0 = y0 - 3;
  const int cx0 = x0 / 2 - 2, cy0 = y0 / 2 - 1;  // coarse staging origin
  const int n0 = f.n0, n1 = f.n1;
  const R om1 = R(1) - omega;
  const int ia = gx0 + 2 * lane, ib = ia + 1;  // ia even
  const bool ina = ia >= 1 && ia <= n0 - 2;
  const bool inb = ib >= 1 && ib <= n0 - 2;
  // column a (even) is red in this wave's rows iff j is even
  const bool ared = ((gy0 + wv) & 1) == 0;
  const bool inR = ared ? ina : inb, inBk = ared ? inb : ina;
  const int iR = ared ? ia : ib, iBk = ared ? ib : ia;
  const cplx<R> xmR = inR ? f.cm0[iR] : zero_c<R>(), xpR = inR ? f.cp0[iR] : zero_c<R>();
  const cplx<R> xmB = inBk ? f.cm0[iBk] : zero_c<R>(), xpB = inBk ? f.cp0[iBk] : zero_c<R>();

  // interior rows of the staged window through buffer resources: halo and
  // boundary nodes read as 0
  const int jl = min(max(gy0, 1), n1 - 1), jh = min(max(gy0 + WY, 1), n1 - 1);
  const __amdgpu_buffer_rsrc_t rb = rows_rsrc(b, jl, jh, n0), rk = rows_rsrc(f.k2, jl, jh, n0);
  const uint32_t obR = col_off<cplx<R>>(inR, iR), obB = col_off<cplx<R>>(inBk, iBk);
  const uint32_t okR = col_off<R>(inR, iR), okB = col_off<R>(inBk, iBk);

  cplx<R> vR[RPW], vB[RPW], bR[RPW], bB[RPW], dR[RPW], dB[RPW], cym[RPW], cyp[RPW];
  R kR[RPW], kB[RPW];
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    const int j = gy0 + ly;
    const bool yin = ly < WY && j >= 1 && j <= n1 - 2;
    const int jc = yin ? j : 1;
    cym[r] = yin ? f.cm1[jc] : zero_c<R>();
    cyp[r] = yin ? f.cp1[jc] : zero_c<R>();
    const uint32_t qb = row_off<cplx<R>>(j - jl, n0), qk = row_off<R>(j - jl, n0);
    bR[r] = ld_c(rb, obR + qb, cplx<R>());
    bB[r] = ld_c(rb, obB + qb, cplx<R>());
    kR[r] = ld_r(rk, okR + qk, R());
    kB[r] = ld_r(rk, okB + qk, R());
  }
  for (int q = threadIdx.x; q < CWY * CWX; q += NT) {
    const int cy = q / CWX, cx = q % CWX;
    const int I = cx0 + cx, J = cy0 + cy;
    se[cy][cx] = (I >= 0 && I < c.n0 && J >= 0 && J < c.n1) ? ec[(int64_t)J * c.n0 + I] : zero_c<R>();
  }
  // inverse diagonals and the down pass's zero-guess red relaxation
  // t = w b / D (0 off the interior)
  // Row conditions depend on the wave (uniform) and are tested apart from the
  // lane conditions, so the compiler branches on them instead of carrying a
  // per-lane exit state through the unrolled row loops.
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    if (ly < WY) {
      const int j = gy0 + ly;
      const bool yin = j >= 1 && j <= n1 - 2;
      dR[r] = (yin && inR) ? inv_cycle(xmR + xpR + cym[r] + cyp[r] + (kR[r] * f.beta + f.c)) : zero_c<R>();
      dB[r] = (yin && inBk) ? inv_cycle(xmB + xpB + cym[r] + cyp[r] + (kB[r] * f.beta + f.c)) : zero_c<R>();
      vR[r] = omega * (bR[r] * dR[r]);
      sR[ly][lane] = vR[r];
    }
  }
  __syncthreads();
  // the down pass's black relaxation t = w (b + o) / D on rings 2 and
  // closer (its red neighbours: own pair, the pair on the other side, own
  // pair one row up and down), then v = t + P ec (bilinear in index space;
  // column a is even: its correction is se[cj][lane] (j even) or the mean
  // over rows cj, cj + 1 (j odd); column b adds the neighbour column).
  // Black values to LDS; red ones stay in registers.
  const int side = ared ? 1 : -1;  // pair holding a node's neighbour of the other colour across the pair
  const int ps = lane + side;
  const bool pin = ps >= 0 && ps < 64;
  const int psc = pin ? ps : lane;
  const cplx<R> wBo = ared ? xmB : xpB, wBn = ared ? xpB : xmB;  // black node: own-pair / other-pair weights
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    vB[r] = zero_c<R>();
    if (ly >= 1 && ly <= WY - 2) {  // ring 3: red t only
      const int j = gy0 + ly;
      const bool yin = j >= 1 && j <= n1 - 2;
      if (pin) {
        const cplx<R> tb =
            bB[r] + (wBo * sR[ly][lane] + wBn * sR[ly][psc] + cym[r] * sR[ly - 1][lane] + cyp[r] * sR[ly + 1][lane]);
        vB[r] = omega * (tb * dB[r]);
      }
      if (yin) {
        const int cj = (j >> 1) - cy0;
        cplx<R> pa, pb;
        if ((j & 1) == 0) {
          pa = se[cj][lane];
          pb = R(0.5) * (se[cj][lane] + se[cj][lane + 1]);
        } else {
          pa = R(0.5) * (se[cj][lane] + se[cj + 1][lane]);
          pb = R(0.25) * (se[cj][lane] + se[cj][lane + 1] + se[cj + 1][lane] + se[cj + 1][lane + 1]);
        }
        if (inR) vR[r] = vR[r] + (ared ? pa : pb);
        if (inBk) vB[r] = vB[r] + (ared ? pb : pa);
      }
      sB[ly][lane] = vB[r];
    }
  }
  __syncthreads();
  // red relaxation on the tile plus a one-node ring.  The red node's black
  // neighbours: own black and the black of pair lane - side in its row (red
  // in column a: left = black of lane - 1), own black one row up and down.
  const int qs = lane - side;
  const bool qin = qs >= 0 && qs < 64;
  const int pq = qin ? qs : lane;
  const cplx<R> wRo = ared ? xpR : xmR, wRn = ared ? xmR : xpR;  // own-pair / other-pair neighbour weights
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    const int j = gy0 + ly;
    if (ly >= 2 && ly <= WY - 3 && j >= 1 && j <= n1 - 2) {
      if (qin && inR) {
        const cplx<R> o =
            wRo * sB[ly][lane] + wRn * sB[ly][pq] + cym[r] * sB[ly - 1][lane] + cyp[r] * sB[ly + 1][lane];
        vR[r] = om1 * vR[r] + omega * ((bR[r] + o) * dR[r]);
        sR[ly][lane] = vR[r];
      }
    }
  }
  __syncthreads();
  // black relaxation on the owned tile (pairs 2..61, rows 3..TY+2); write
  // both nodes of every owned pair
  const bool own_x = lane >= 2 && lane <= 61;
  const uint32_t osR = col_off<cplx<R>>(own_x && iR < n0, iR), osB = col_off<cplx<R>>(own_x && iBk < n0, iBk);
  const __amdgpu_buffer_rsrc_t ro = rows_rsrc(u_out, y0, min(y0 + TY, n1), n0);
#pragma unroll
  for (int r = 0; r < RPW; r++) {
    const int ly = wv + 4 * r;
    const int j = gy0 + ly;
    if (ly >= 3 && ly < TY + 3 && j < n1) {
      cplx<R> outB = vB[r];
      if (own_x && inBk && j >= 1 && j <= n1 - 2) {
        const cplx<R> o =
            wBo * sR[ly][lane] + wBn * sR[ly][psc] + cym[r] * sR[ly - 1][lane] + cyp[r] * sR[ly + 1][lane];
        outB = om1 * outB + omega * ((bB[r] + o) * dB[r]);
      }
      const uint32_t qo = row_off<cplx<R>>(j - y0, n0);
      st_c(ro, osR + qo, vR[r]);
      st_c(ro, osB + qo, outB);
    }
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
// row-major order.  The node of unknown c (interior row c / ni, column
// c % ni) comes from a float reciprocal, not an integer division: exact here
// (c < 1024, so the product stays more than 0.5 / ni away from an integer).
template <typename R, typename M>
__device__ __forceinline__ void tail_dense(int nu, int tpr, const M *mi, const cplx<R> *b, cplx<R> *x, int n0) {
  const int tid = threadIdx.x, ni = n0 - 2, rows_per_pass = TT / tpr;
  const float inv = 1.0f / (float)ni;
  auto node = [&](int c) {
    const int r = (int)(((float)c + 0.5f) * inv);
    return (r + 1) * n0 + (c - r * ni) + 1;
  };
  for (int r0 = 0; r0 < nu; r0 += rows_per_pass) {
    const int rr = r0 + tid / tpr;
    cplx<R> acc = zero_c<R>();
    if (rr < nu) {
#pragma unroll 4
      for (int c = tid % tpr; c < nu; c += tpr) acc = acc + mi[(int64_t)c * nu + rr] * b[node(c)];
    }
    for (int m = tpr >> 1; m >= 1; m >>= 1) {
      acc.re += __shfl_xor(acc.re, m, 64);
      acc.im += __shfl_xor(acc.im, m, 64);
    }
    if (rr < nu && tid % tpr == 0) x[node(rr)] = acc;
  }
}

template <typename R, bool MR>
__global__ __launch_bounds__(TT) void k_tail(TailArgs<R> a, RhsSet rs) {
  __shared__ TailLds<R> S;
  const int tid = threadIdx.x;
  // one workgroup per right-hand side (the kernel argument block is not written)
  const int64_t rq = MR ? rhs_index(rs) * rhs_stride((int64_t)a.g[0].n0 * a.g[0].n1) : 0;
  const cplx<R> *const b0 = a.b0 + rq;
  cplx<R> *const u0 = a.u0 + rq;
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
      // row from a float reciprocal (exact: p < kTailCap)
      const int j = (int)(((float)p + 0.5f) * (1.0f / (float)g.n0)), i = p - j * g.n0;
      lv[sl] = P < a.poff[a.nl] && p0 < nn ? k : -1;
      pv[sl] = p;
      cxm[sl] = g.cm0[i];
      cxp[sl] = g.cp0[i];
      cym[sl] = g.cm1[j];
      cyp[sl] = g.cp1[j];
      kv[sl] = g.k2[p];
      bv[sl] = b0[k == 0 ? p : 0];
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
      const int p = pv[sl], j = (int)(((float)p + 0.5f) * (1.0f / (float)g.n0)), i = p - j * g.n0;
      const int P = a.noff[kk] + p;
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

  // Colour phases enumerate node pairs (columns 2h, 2h + 1 of a row: one red,
  // one black), so every thread has one node of the colour at hand; row
  // indices come from a float reciprocal (exact for these sizes: the error is
  // far below the half-node margin), not an integer division.
  // down: black relaxation, red residual, restriction (which also performs
  // the next level's zero-guess red relaxation on the nodes it produces)
  for (int k = 0; k < last; k++) {
    const Grid<R> &g = a.g[k];
    const int n0 = g.n0, n1 = g.n1, no = a.noff[k], wo = a.woff[k];
    const int H = (n0 + 1) >> 1, np = n1 * H;
    const float invH = 1.0f / (float)H;
    const cplx<R> *xm = S.xm + wo, *xp = S.xp + wo, *ym = S.ym + wo, *yp = S.yp + wo;
    cplx<R> *b = S.b + no, *t = S.t + no, *w = S.w + no, *d = S.d + no;
    for (int q = tid; q < np; q += TT) {
      const int j = (int)(((float)q + 0.5f) * invH), i = 2 * (q - j * H) + ((j + 1) & 1);  // black
      if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
        const int p = j * n0 + i;
        const cplx<R> tb = b[p] + (xm[i] * t[p - 1] + xp[i] * t[p + 1] + ym[j] * t[p - n0] + yp[j] * t[p + n0]);
        t[p] = om * (tb * d[p]);
        w[p] = om1 * tb;  // black residual (1 - w)(b + o)
      }
    }
    __syncthreads();
    // red residual (1 - w) b + o; only interior residuals are read below
    for (int q = tid; q < np; q += TT) {
      const int j = (int)(((float)q + 0.5f) * invH), i = 2 * (q - j * H) + (j & 1);  // red
      if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
        const int p = j * n0 + i;
        w[p] = om1 * b[p] + (xm[i] * t[p - 1] + xp[i] * t[p + 1] + ym[j] * t[p - n0] + yp[j] * t[p + n0]);
      }
    }
    __syncthreads();
    const Grid<R> &gc = a.g[k + 1];
    const int c0 = gc.n0, nc = c0 * gc.n1, nco = a.noff[k + 1];
    const float inv0 = 1.0f / (float)c0;
    for (int q = tid; q < nc; q += TT) {
      const int J = (int)(((float)q + 0.5f) * inv0), I = q - J * c0;
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

  // dense solve on the coarsest level; its boundary nodes (read as 0 by the
  // prolongation) are cleared by other threads in the same phase: the solve
  // writes only interior nodes
  {
    const Grid<R> &g = a.g[last];
    const int nn = g.n0 * g.n1, no = a.noff[last];
    const float inv0 = 1.0f / (float)g.n0;
    for (int p = tid; p < nn; p += TT) {
      const int j = (int)(((float)p + 0.5f) * inv0), i = p - j * g.n0;
      if (i == 0 || i == g.n0 - 1 || j == 0 || j == g.n1 - 1) S.w[no + p] = zero_c<R>();
    }
    if (minv_lds) tail_dense(a.nunk, a.tpr, S.mi, S.b + no, S.w + no, g.n0);
    else tail_dense(a.nunk, a.tpr, a.minvT, S.b + no, S.w + no, g.n0);
    __syncthreads();
  }

  // up: prolongation + correction, then the red-black post-sweep in place;
  // the first level's black sweep writes the result (both nodes of every
  // pair) to global memory
  for (int k = last - 1; k >= 0; k--) {
    const Grid<R> &g = a.g[k];
    const int n0 = g.n0, n1 = g.n1, no = a.noff[k], wo = a.woff[k];
    const int H = (n0 + 1) >> 1, np = n1 * H;
    const float invH = 1.0f / (float)H;
    const int c0 = a.g[k + 1].n0;
    const cplx<R> *xm = S.xm + wo, *xp = S.xp + wo, *ym = S.ym + wo, *yp = S.yp + wo;
    const cplx<R> *b = S.b + no, *t = S.t + no, *d = S.d + no, *e = S.w + a.noff[k + 1];
    cplx<R> *w = S.w + no;
    for (int q = tid; q < np; q += TT) {
      const int j = (int)(((float)q + 0.5f) * invH), i0 = 2 * (q - j * H);
      const bool yin = j >= 1 && j <= n1 - 2;
      const cplx<R> *e0 = e + (j >> 1) * c0 + (i0 >> 1);  // i0 even: coarse column i0 / 2
      // column i0 (even): coarse node or the mean over two coarse rows
      cplx<R> pa = zero_c<R>(), pb = zero_c<R>();
      if (yin) {
        if ((j & 1) == 0) {
          pa = e0[0];
          pb = R(0.5) * (e0[0] + e0[1]);
        } else {
          pa = R(0.5) * (e0[0] + e0[c0]);
          pb = R(0.25) * (e0[0] + e0[1] + e0[c0] + e0[c0 + 1]);
        }
      }
      const int p = j * n0 + i0;
      w[p] = (yin && i0 >= 1 && i0 <= n0 - 2) ? t[p] + pa : zero_c<R>();
      if (i0 + 1 < n0) w[p + 1] = (yin && i0 + 1 <= n0 - 2) ? t[p + 1] + pb : zero_c<R>();
    }
    __syncthreads();
    for (int colour = 0; colour < 2; colour++) {
      for (int q = tid; q < np; q += TT) {
        const int j = (int)(((float)q + 0.5f) * invH), h2 = 2 * (q - j * H);
        const int i = h2 + ((j + colour) & 1);  // the pair's node of this colour
        const int p = j * n0 + i;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
          const cplx<R> o = xm[i] * w[p - 1] + xp[i] * w[p + 1] + ym[j] * w[p - n0] + yp[j] * w[p + n0];
          w[p] = om1 * w[p] + om * ((b[p] + o) * d[p]);
        }
        if (k == 0 && colour == 1) {
          const int pp = j * n0 + h2;  // both nodes of the pair (the red one is final)
          u0[pp] = w[pp];
          if (h2 + 1 < n0) u0[pp + 1] = w[pp + 1];
        }
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ wide tail
// The same cycle as k_tail (FP32) from a level of up to 65^2 nodes.  To fit
// a workgroup's 160 KiB of LDS a node keeps its right-hand side, iterate,
// residual and k^2 (28 B) and its inverse diagonal is formed where it is used,
// from the LDS weights and k^2 by k_tail's set-up expression (the same value);
// the coarsest inverse is read from memory.  The set-up loads the weights
// (wave k: level k's, two entries per lane), k^2 of every node and the first
// level's right-hand side; the first level's zero-guess red relaxation is a
// phase of its own.
struct TailLdsWide {
  cplx<float> xm[kTailWideWeights], xp[kTailWideWeights], ym[kTailWideWeights], yp[kTailWideWeights];
  cplx<float> b[kTailWideCap], t[kTailWideCap], w[kTailWideCap];
  float k[kTailWideCap];
};
static_assert(sizeof(TailLdsWide) <= 163840, "the wide tail's vectors fit a workgroup's LDS");

template <bool MR>
__global__ __launch_bounds__(TT) void k_tail_wide(TailArgs<float> a, RhsSet rs) {
  __shared__ TailLdsWide S;
  const int tid = threadIdx.x;
  const int64_t rq = MR ? rhs_index(rs) * rhs_stride((int64_t)a.g[0].n0 * a.g[0].n1) : 0;
  const cplx<float> *const b0 = a.b0 + rq;
  cplx<float> *const u0 = a.u0 + rq;
  const float om = a.omega, om1 = 1.0f - a.omega;
  const int last = a.nl - 1;
  // inverse diagonal of node p = (i, j) of level k (k uniform)
  auto dinv = [&](int k, int i, int j, int p) {
    const Grid<float> &g = a.g[k];
    const int wo = a.woff[k];
    return inv_c(S.xm[wo + i] + S.xp[wo + i] + S.ym[wo + j] + S.yp[wo + j] + (S.k[a.noff[k] + p] * g.beta + g.c));
  };
  {
    const int ln = tid & 63;
    const int kw = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (kw < a.nl) {
      const Grid<float> &gw = a.g[kw];
      const int wo = a.woff[kw], nw = a.woff[kw + 1] - wo;
      for (int q = ln; q < nw; q += 64) {
        const int q0 = q < gw.n0 ? q : gw.n0 - 1, q1 = q < gw.n1 ? q : gw.n1 - 1;
        S.xm[wo + q] = gw.cm0[q0];
        S.xp[wo + q] = gw.cp0[q0];
        S.ym[wo + q] = gw.cm1[q1];
        S.yp[wo + q] = gw.cp1[q1];
      }
    }
    // nodes: slot sl of thread tid is padded index P = tid + sl TT (waves
    // never straddle levels, so a wave's level is uniform)
    constexpr int kSlots = (kTailWideCap + kTailMaxLevels * 63 + TT - 1) / TT;
    float kv[kSlots];
    cplx<float> bv[kSlots];
    int lv[kSlots], pv[kSlots];
#pragma unroll
    for (int sl = 0; sl < kSlots; sl++) {
      const int P = tid + sl * TT;
      int k = 0;
      for (int q = 1; q < a.nl; q++) k = P >= a.poff[q] ? q : k;
      k = __builtin_amdgcn_readfirstlane(k);
      const Grid<float> &g = a.g[k];
      const int nn = g.n0 * g.n1;
      const int p0 = P - a.poff[k], p = p0 < nn ? p0 : nn - 1;
      lv[sl] = P < a.poff[a.nl] && p0 < nn ? k : -1;
      pv[sl] = p;
      kv[sl] = g.k2[p];
      bv[sl] = b0[k == 0 ? p : 0];
    }
#pragma unroll
    for (int sl = 0; sl < kSlots; sl++) {
      const int k = lv[sl];
      if (k < 0) continue;
      const int kk = __builtin_amdgcn_readfirstlane(k);
      const Grid<float> &g = a.g[kk];
      const int p = pv[sl], j = (int)(((float)p + 0.5f) * (1.0f / (float)g.n0)), i = p - j * g.n0;
      const int P = a.noff[kk] + p;
      S.k[P] = kv[sl];
      if (kk == 0) S.b[P] = (i >= 1 && i <= g.n0 - 2 && j >= 1 && j <= g.n1 - 2) ? bv[sl] : zero_c<float>();
    }
  }
  __syncthreads();
  {
    // the first level's zero-guess red relaxation t = w b / D (0 elsewhere)
    const Grid<float> &g = a.g[0];
    const int n0 = g.n0, nn = n0 * g.n1;
    const float inv0 = 1.0f / (float)n0;
    for (int p = tid; p < nn; p += TT) {
      const int j = (int)(((float)p + 0.5f) * inv0), i = p - j * n0;
      const bool in = i >= 1 && i <= n0 - 2 && j >= 1 && j <= g.n1 - 2;
      S.t[p] = (in && ((i + j) & 1) == 0) ? om * (S.b[p] * dinv(0, i, j, p)) : zero_c<float>();
    }
  }
  __syncthreads();

  // down: black relaxation, red residual, restriction (with the next level's
  // zero-guess red relaxation), as in k_tail
  for (int k = 0; k < last; k++) {
    const Grid<float> &g = a.g[k];
    const int n0 = g.n0, n1 = g.n1, no = a.noff[k], wo = a.woff[k];
    const int H = (n0 + 1) >> 1, np = n1 * H;
    const float invH = 1.0f / (float)H;
    const cplx<float> *xm = S.xm + wo, *xp = S.xp + wo, *ym = S.ym + wo, *yp = S.yp + wo;
    cplx<float> *b = S.b + no, *t = S.t + no, *w = S.w + no;
    for (int q = tid; q < np; q += TT) {
      const int j = (int)(((float)q + 0.5f) * invH), i = 2 * (q - j * H) + ((j + 1) & 1);  // black
      if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
        const int p = j * n0 + i;
        const cplx<float> tb = b[p] + (xm[i] * t[p - 1] + xp[i] * t[p + 1] + ym[j] * t[p - n0] + yp[j] * t[p + n0]);
        t[p] = om * (tb * dinv(k, i, j, p));
        w[p] = om1 * tb;
      }
    }
    __syncthreads();
    for (int q = tid; q < np; q += TT) {
      const int j = (int)(((float)q + 0.5f) * invH), i = 2 * (q - j * H) + (j & 1);  // red
      if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
        const int p = j * n0 + i;
        w[p] = om1 * b[p] + (xm[i] * t[p - 1] + xp[i] * t[p + 1] + ym[j] * t[p - n0] + yp[j] * t[p + n0]);
      }
    }
    __syncthreads();
    const Grid<float> &gc = a.g[k + 1];
    const int c0 = gc.n0, nc = c0 * gc.n1, nco = a.noff[k + 1];
    const float inv0 = 1.0f / (float)c0;
    for (int q = tid; q < nc; q += TT) {
      const int J = (int)(((float)q + 0.5f) * inv0), I = q - J * c0;
      cplx<float> acc = zero_c<float>(), tv = zero_c<float>();
      if (I >= 1 && I <= c0 - 2 && J >= 1 && J <= gc.n1 - 2) {
        const cplx<float> *r0 = w + (2 * J) * n0 + 2 * I;
        acc = 0.25f * r0[0] + 0.125f * (r0[-1] + r0[1] + r0[-n0] + r0[n0]) +
              0.0625f * (r0[-n0 - 1] + r0[-n0 + 1] + r0[n0 - 1] + r0[n0 + 1]);
        if (((I + J) & 1) == 0) tv = om * (acc * dinv(k + 1, I, J, q));
      }
      S.b[nco + q] = acc;
      S.t[nco + q] = tv;
    }
    __syncthreads();
  }

  // dense solve on the coarsest level (inverse from memory); boundary zeros
  {
    const Grid<float> &g = a.g[last];
    const int nn = g.n0 * g.n1, no = a.noff[last];
    const float inv0 = 1.0f / (float)g.n0;
    for (int p = tid; p < nn; p += TT) {
      const int j = (int)(((float)p + 0.5f) * inv0), i = p - j * g.n0;
      if (i == 0 || i == g.n0 - 1 || j == 0 || j == g.n1 - 1) S.w[no + p] = zero_c<float>();
    }
    tail_dense(a.nunk, a.tpr, a.minvT, S.b + no, S.w + no, g.n0);
    __syncthreads();
  }

  // up: prolongation + correction, then the red-black post-sweep, as in k_tail
  for (int k = last - 1; k >= 0; k--) {
    const Grid<float> &g = a.g[k];
    const int n0 = g.n0, n1 = g.n1, no = a.noff[k], wo = a.woff[k];
    const int H = (n0 + 1) >> 1, np = n1 * H;
    const float invH = 1.0f / (float)H;
    const int c0 = a.g[k + 1].n0;
    const cplx<float> *xm = S.xm + wo, *xp = S.xp + wo, *ym = S.ym + wo, *yp = S.yp + wo;
    const cplx<float> *b = S.b + no, *t = S.t + no, *e = S.w + a.noff[k + 1];
    cplx<float> *w = S.w + no;
    for (int q = tid; q < np; q += TT) {
      const int j = (int)(((float)q + 0.5f) * invH), i0 = 2 * (q - j * H);
      const bool yin = j >= 1 && j <= n1 - 2;
      const cplx<float> *e0 = e + (j >> 1) * c0 + (i0 >> 1);
      cplx<float> pa = zero_c<float>(), pb = zero_c<float>();
      if (yin) {
        if ((j & 1) == 0) {
          pa = e0[0];
          pb = 0.5f * (e0[0] + e0[1]);
        } else {
          pa = 0.5f * (e0[0] + e0[c0]);
          pb = 0.25f * (e0[0] + e0[1] + e0[c0] + e0[c0 + 1]);
        }
      }
      const int p = j * n0 + i0;
      w[p] = (yin && i0 >= 1 && i0 <= n0 - 2) ? t[p] + pa : zero_c<float>();
      if (i0 + 1 < n0) w[p + 1] = (yin && i0 + 1 <= n0 - 2) ? t[p + 1] + pb : zero_c<float>();
    }
    __syncthreads();
    for (int colour = 0; colour < 2; colour++) {
      for (int q = tid; q < np; q += TT) {
        const int j = (int)(((float)q + 0.5f) * invH), h2 = 2 * (q - j * H);
        const int i = h2 + ((j + colour) & 1);
        const int p = j * n0 + i;
        if (i >= 1 && i <= n0 - 2 && j >= 1 && j <= n1 - 2) {
          const cplx<float> o = xm[i] * w[p - 1] + xp[i] * w[p + 1] + ym[j] * w[p - n0] + yp[j] * w[p + n0];
          w[p] = om1 * w[p] + om * ((b[p] + o) * dinv(k, i, j, p));
        }
        if (k == 0 && colour == 1) {
          const int pp = j * n0 + h2;
          u0[pp] = w[pp];
          if (h2 + 1 < n0) u0[pp + 1] = w[pp + 1];
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace

// The tile height of the fused kernels is a launch parameter chosen by the
// host (autotuned per grid size and dtype): coarse rows per down block in
// {2, ..., 6, 8, 16} (16 only in FP32, whose tile fits the LDS), fine rows
// per up block in {4, 8, 10, 12, 16, 32}.
template <typename R, int SRC, bool MR>
void launch_down_mr(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, const DownSrc<R> &src, cplx<R> *rc,
                    R omega, int rows, hipStream_t s, const RhsSet &rs) {
  constexpr int CX = 61;
  const int tx = (coarse.n0 + CX - 1) / CX;
  const int tiles = tx * ((coarse.n1 + rows - 1) / rows);
  const dim3 grid(xcd_padded(tiles), rs.count), block(NT);
  switch (rows) {
    case 2: launch_k((k_down_rb<R, 2, SRC, MR>), grid, block, 0, s, fine, coarse, b, src, rc, omega, tx, tiles, rs); break;
    case 3: launch_k((k_down_rb<R, 3, SRC, MR>), grid, block, 0, s, fine, coarse, b, src, rc, omega, tx, tiles, rs); break;
    case 4: launch_k((k_down_rb<R, 4, SRC, MR>), grid, block, 0, s, fine, coarse, b, src, rc, omega, tx, tiles, rs); break;
    case 5: launch_k((k_down_rb<R, 5, SRC, MR>), grid, block, 0, s, fine, coarse, b, src, rc, omega, tx, tiles, rs); break;
    case 6: launch_k((k_down_rb<R, 6, SRC, MR>), grid, block, 0, s, fine, coarse, b, src, rc, omega, tx, tiles, rs); break;
    case 16:
      if constexpr (sizeof(R) == 4) {
        launch_k((k_down_rb<R, 16, SRC, MR>), grid, block, 0, s, fine, coarse, b, src, rc, omega, tx, tiles, rs);
        break;
      }
      [[fallthrough]];
    default:
      launch_k((k_down_rb<R, 8, SRC, MR>), grid, block, 0, s, fine, coarse, b, src, rc, omega, tx, tiles, rs);
      break;
  }
}

template <typename R, int SRC>
void launch_down(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, const DownSrc<R> &src, cplx<R> *rc,
                 R omega, int rows, hipStream_t s, const RhsSet &rs) {
  if (multi_rhs(rs)) launch_down_mr<R, SRC, true>(fine, coarse, b, src, rc, omega, rows, s, rs);
  else launch_down_mr<R, SRC, false>(fine, coarse, b, src, rc, omega, rows, s, rs);
}

template <typename R>
void launch_down_rb(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, cplx<R> *rc, R omega, int rows,
                    hipStream_t s, const RhsSet &rs) {
  launch_down<R, kDownSrcB>(fine, coarse, b, DownSrc<R>{}, rc, omega, rows, s, rs);
}

template <typename R>
void launch_down_rb_src(const Grid<R> &fine, const Grid<R> &coarse, const DownSrc<R> &src, cplx<R> *rc, R omega,
                        int rows, hipStream_t s) {
  if (src.mode == kDownSrcP) launch_down<R, kDownSrcP>(fine, coarse, nullptr, src, rc, omega, rows, s, one_rhs());
  else launch_down<R, kDownSrcS>(fine, coarse, nullptr, src, rc, omega, rows, s, one_rhs());
}

template <typename R, bool MR>
void launch_up_mr(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, const cplx<R> *ec, cplx<R> *u_out,
                  R omega, int rows, hipStream_t s, const RhsSet &rs) {
  constexpr int TX = 120;
  const int tx = (fine.n0 + TX - 1) / TX;
  const int tiles = tx * ((fine.n1 + rows - 1) / rows);
  const dim3 grid(xcd_padded(tiles), rs.count), block(NT);
  switch (rows) {
    case 4: launch_k((k_up_rb<R, 4, MR>), grid, block, 0, s, fine, coarse, b, ec, u_out, omega, tx, tiles, rs); break;
    case 8: launch_k((k_up_rb<R, 8, MR>), grid, block, 0, s, fine, coarse, b, ec, u_out, omega, tx, tiles, rs); break;
    case 10: launch_k((k_up_rb<R, 10, MR>), grid, block, 0, s, fine, coarse, b, ec, u_out, omega, tx, tiles, rs); break;
    case 12: launch_k((k_up_rb<R, 12, MR>), grid, block, 0, s, fine, coarse, b, ec, u_out, omega, tx, tiles, rs); break;
    case 32: launch_k((k_up_rb<R, 32, MR>), grid, block, 0, s, fine, coarse, b, ec, u_out, omega, tx, tiles, rs); break;
    default: launch_k((k_up_rb<R, 16, MR>), grid, block, 0, s, fine, coarse, b, ec, u_out, omega, tx, tiles, rs); break;
  }
}

template <typename R>
void launch_up_rb(const Grid<R> &fine, const Grid<R> &coarse, const cplx<R> *b, const cplx<R> *ec, cplx<R> *u_out,
                  R omega, int rows, hipStream_t s, const RhsSet &rs) {
  if (multi_rhs(rs)) launch_up_mr<R, true>(fine, coarse, b, ec, u_out, omega, rows, s, rs);
  else launch_up_mr<R, false>(fine, coarse, b, ec, u_out, omega, rows, s, rs);
}

template <typename R>
void launch_tail(const TailArgs<R> &a, hipStream_t s, const RhsSet &rs) {
  if constexpr (sizeof(R) == 4) {
    // beyond k_tail's capacity (or a level wider than one wave): the wide tail
    if (a.noff[a.nl] > kTailCap || a.g[0].n0 > 64 || a.g[0].n1 > 64) {
      if (multi_rhs(rs)) launch_k((k_tail_wide<true>), dim3(1, rs.count), dim3(TT), 0, s, a, rs);
      else launch_k((k_tail_wide<false>), dim3(1, 1), dim3(TT), 0, s, a, rs);
      return;
    }
  }
  if (multi_rhs(rs)) launch_k((k_tail<R, true>), dim3(1, rs.count), dim3(TT), 0, s, a, rs);
  else launch_k((k_tail<R, false>), dim3(1, 1), dim3(TT), 0, s, a, rs);
}

template void launch_down_rb<double>(const Grid<double> &, const Grid<double> &, const cplx<double> *, cplx<double> *,
                                     double, int, hipStream_t, const RhsSet &);
template void launch_down_rb<float>(const Grid<float> &, const Grid<float> &, const cplx<float> *, cplx<float> *,
                                    float, int, hipStream_t, const RhsSet &);
template void launch_up_rb<double>(const Grid<double> &, const Grid<double> &, const cplx<double> *,
                                   const cplx<double> *, cplx<double> *, double, int, hipStream_t, const RhsSet &);
template void launch_down_rb_src<float>(const Grid<float> &, const Grid<float> &, const DownSrc<float> &, cplx<float> *,
                                        float, int, hipStream_t);
template void launch_down_rb_src<double>(const Grid<double> &, const Grid<double> &, const DownSrc<double> &,
                                         cplx<double> *, double, int, hipStream_t);
template void launch_tail<double>(const TailArgs<double> &, hipStream_t, const RhsSet &);
template void launch_tail<float>(const TailArgs<float> &, hipStream_t, const RhsSet &);
template void launch_up_rb<float>(const Grid<float> &, const Grid<float> &, const cplx<float> *, const cplx<float> *,
                                  cplx<float> *, float, int, hipStream_t, const RhsSet &);

}  // namespace ecs
