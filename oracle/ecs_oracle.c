/*
 * ecs_oracle.c -- plain FP64 CPU reference of the ECS Helmholtz solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the GPU
 * path.  Every routine is a direct, unblocked, unfused transcription of the
 * definition it cites (bin Zubair, Reps, Vanroose, "A preconditioned iterative
 * solver for the scattering solutions of the Schroedinger equation"):
 *
 *   Sec. 3.1        exterior complex scaling: z(x) = x inside, rotated contour
 *                   z = s + (x - s) e^{i theta} beyond the layer start s.
 *   Sec. 3.2        3-point second difference on a non-uniform (complex) grid,
 *                   tensor-summed to 2D / 3D; homogeneous Dirichlet at the end
 *                   of every contour.
 *   Sec. 4.1 / 5    preconditioner operators: CSL  -Lap + (b1 + i b2) k^2,
 *                   CSG  Z on the grid rotated by e^{i theta_alpha},
 *                   QD   (1 - i) I + Z / |Re lambda0|.
 *   Sec. 4.2        Algorithm 1 (multigrid with cycle indices gamma_f,
 *                   gamma_c), omega-Jacobi and red-black SOR smoothers,
 *                   full-weighting restriction, bilinear prolongation,
 *                   rediscretised coarse operators, exact coarsest solve.
 *   Sec. 5          right-preconditioned Krylov outer solvers (Bi-CGSTAB;
 *                   GMRES / restarted GMRES; flexible GMRES).
 *
 * Parity pins: every function here is checked in tests/test_oracle_*.py
 * against closed forms or brute force (Lemma 3.1 spectrum, uniform-grid
 * Laplacian eigenvalues, the symmetry of W*A, the QD disk of Sec. 4.1, a
 * manufactured solution, dense LU, textbook SOR / two-grid matrix forms,
 * multigrid visit counts).  No function is "parity unpinned".
 *
 * Conventions: nodes per axis n[a] include both Dirichlet end nodes; arrays are
 * node-major with x fastest, idx = (k*n1 + j)*n0 + i; 2D problems have n[2]=1.
 * Boundary nodes of every vector are kept at zero.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORA_MAXLEV 16

/* ---------------------------------------------------------------- levels -- */

typedef struct {
  int n[3];          /* nodes per axis (n[2] = 1 in 2D)                        */
  int64_t nn;        /* total nodes                                            */
  cplx *z[3];        /* complex node coordinates along each axis               */
  /* second-difference weights of the original grid (operator A = L - k^2)   */
  cplx *am[3], *ap[3], *w[3];
  /* weights of the preconditioner grid (rotated for CSG, else the same)       */
  cplx *mm[3], *mp[3];
  double *k2;        /* k^2 at the real node coordinates                       */
  cplx *b, *u, *r;   /* per-level work vectors for the multigrid recursion     */
  /* coarsest level: dense LU of the preconditioner operator on interior nodes */
  int nunk;
  cplx *lu;
  int *piv;
  int64_t *unk;      /* interior unknown -> node index                         */
} olevel;

typedef struct {
  int dim;
  int nlev;
  olevel lev[ORA_MAXLEV];
  /* preconditioner operator M = alpha * L_M + (beta k^2 + c) I              */
  cplx alpha, beta, c;
  int kind;          /* 0 none(A itself), 1 Laplace, 2 CSL, 3 CSG, 4 QD        */
  double p1, p2;     /* kind parameters (CSL b1,b2 | CSG theta_alpha | QD lam)  */
  /* multigrid schedule                                                      */
  int smoother;      /* 0 omega-Jacobi, 1 red-black SOR                         */
  double omega;
  int nu1, nu2, gf, gc;
  int64_t visits[ORA_MAXLEV];
  int64_t cycles;    /* number of top-level multigrid applications            */
  int nthreads_used;
} ohier;

static int active(const olevel *L, int a) { return L->n[a] > 1; }

static void *xcalloc(size_t n, size_t s) {
  void *p = calloc(n ? n : 1, s);
  if (!p) { fprintf(stderr, "ecs_oracle: out of memory\n"); abort(); }
  return p;
}

/* Sec. 3.1: nodal ECS map.  Real nodes x_i = lo + i (hi - lo)/(n - 1); beyond
 * the layer start s on a flagged side the coordinate is rotated into the
 * complex plane, z = s + (x - s) e^{i theta}, so every complex cell has the
 * real length of its real counterpart times e^{i theta}. */
void ora_zmap(int n, double lo, double hi, int ecs_lo, double s_lo, double th_lo,
              int ecs_hi, double s_hi, double th_hi, double *z_out /* 2n */) {
  for (int i = 0; i < n; i++) {
    double x = (n > 1) ? lo + (double)i * (hi - lo) / (double)(n - 1) : lo;
    cplx z = x;
    if (ecs_hi && x > s_hi) z = s_hi + (x - s_hi) * cexp(I * th_hi);
    if (ecs_lo && x < s_lo) z = s_lo + (x - s_lo) * cexp(I * th_lo);
    z_out[2 * i] = creal(z);
    z_out[2 * i + 1] = cimag(z);
  }
}

/* Sec. 3.2: weights of the non-uniform second difference at node i,
 *   -u'' ~ a-_i (u_i - u_{i-1}) + a+_i (u_i - u_{i+1}),
 *   a-_i = 2 / ((h_{i-1} + h_i) h_{i-1}),  a+_i = 2 / ((h_{i-1} + h_i) h_i),
 * with h_j = z_{j+1} - z_j.  w_i = (h_{i-1} + h_i)/2 is the dual cell width
 * (the symmetriser: w_i a+_i = w_{i+1} a-_{i+1} = 1/h_i).  End nodes get 0. */
static void second_diff_weights(int n, const cplx *z, cplx *am, cplx *ap, cplx *w) {
  for (int i = 0; i < n; i++) { am[i] = 0; ap[i] = 0; if (w) w[i] = 1; }
  for (int i = 1; i + 1 < n; i++) {
    cplx hm = z[i] - z[i - 1], hp = z[i + 1] - z[i];
    am[i] = 2.0 / ((hm + hp) * hm);
    ap[i] = 2.0 / ((hm + hp) * hp);
    if (w) w[i] = 0.5 * (hm + hp);
  }
}

static int64_t idx3(const olevel *L, int i, int j, int k) {
  return ((int64_t)k * L->n[1] + j) * L->n[0] + i;
}

static int interior(const olevel *L, int a, int i) {
  return active(L, a) ? (i >= 1 && i <= L->n[a] - 2) : (i == 0);
}

static int64_t stride(const olevel *L, int a) {
  return a == 0 ? 1 : (a == 1 ? L->n[0] : (int64_t)L->n[0] * L->n[1]);
}

/* ------------------------------------------------------------- operators -- */

/* (L u)_p with the given 1D weights: the tensor sum of the 1D second
 * differences over the active axes (Sec. 3.2). */
static cplx lap_at(const olevel *L, cplx *const wm[3], cplx *const wp[3],
                   const cplx *u, int i, int j, int k) {
  int c[3] = {i, j, k};
  int64_t p = idx3(L, i, j, k);
  cplx s = 0;
  for (int a = 0; a < 3; a++) {
    if (!active(L, a)) continue;
    int64_t st = stride(L, a);
    s += wm[a][c[a]] * (u[p] - u[p - st]) + wp[a][c[a]] * (u[p] - u[p + st]);
  }
  return s;
}

/* (A u)_p = (L u)_p - k^2_p u_p : the discrete ECS Helmholtz operator Z. */
static cplx A_at(const olevel *L, const cplx *u, int i, int j, int k) {
  int64_t p = idx3(L, i, j, k);
  return lap_at(L, L->am, L->ap, u, i, j, k) - L->k2[p] * u[p];
}

/* (M u)_p = alpha (L_M u)_p + (beta k^2_p + c) u_p : the preconditioner. */
static cplx M_at(const ohier *H, const olevel *L, const cplx *u, int i, int j, int k) {
  int64_t p = idx3(L, i, j, k);
  return H->alpha * lap_at(L, L->mm, L->mp, u, i, j, k) + (H->beta * L->k2[p] + H->c) * u[p];
}

/* diagonal entry of M at p */
static cplx M_diag(const ohier *H, const olevel *L, int i, int j, int k) {
  int c[3] = {i, j, k};
  cplx s = 0;
  for (int a = 0; a < 3; a++)
    if (active(L, a)) s += L->mm[a][c[a]] + L->mp[a][c[a]];
  return H->alpha * s + H->beta * L->k2[idx3(L, i, j, k)] + H->c;
}

/* (A^T y)_p built from the explicitly transposed stencil: the entry of A in
 * row q, column p is read off row q's weights, so
 *   (A^T y)_p = sum_a [ (a-_p + a+_p) y_p - a+_{p-1} y_{p-1} - a-_{p+1} y_{p+1} ]
 *               - k^2_p y_p
 * (neighbours q on the boundary carry no row, their y is zero). */
static cplx AT_at(const olevel *L, const cplx *y, int i, int j, int k) {
  int c[3] = {i, j, k};
  int64_t p = idx3(L, i, j, k);
  cplx s = 0;
  for (int a = 0; a < 3; a++) {
    if (!active(L, a)) continue;
    int64_t st = stride(L, a);
    int ia = c[a];
    s += (L->am[a][ia] + L->ap[a][ia]) * y[p];
    if (interior(L, a, ia - 1)) s -= L->ap[a][ia - 1] * y[p - st];
    if (interior(L, a, ia + 1)) s -= L->am[a][ia + 1] * y[p + st];
  }
  return s - L->k2[p] * y[p];
}

#define FOR_INTERIOR(L, i, j, k)                                              \
  for (int k = active(L, 2) ? 1 : 0; k < (active(L, 2) ? (L)->n[2] - 1 : 1); k++) \
    for (int j = 1; j < (L)->n[1] - 1; j++)                                   \
      for (int i = 1; i < (L)->n[0] - 1; i++)

static void zero_vec(cplx *v, int64_t n) { memset(v, 0, sizeof(cplx) * (size_t)n); }

/* which: 0 -> A, 1 -> M, 2 -> A^T */
static void apply_level(const ohier *H, const olevel *L, int which, const cplx *x, cplx *y) {
  zero_vec(y, L->nn);
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = active(L, 2) ? 1 : 0; k < (active(L, 2) ? L->n[2] - 1 : 1); k++)
    for (int j = 1; j < L->n[1] - 1; j++)
      for (int i = 1; i < L->n[0] - 1; i++) {
        cplx v = which == 0 ? A_at(L, x, i, j, k)
               : which == 1 ? M_at(H, L, x, i, j, k)
                            : AT_at(L, x, i, j, k);
        y[idx3(L, i, j, k)] = v;
      }
}

/* r = b - M u on level L (interior; boundary r = 0) */
static void residual_level(const ohier *H, const olevel *L, const cplx *b, const cplx *u, cplx *r) {
  zero_vec(r, L->nn);
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = active(L, 2) ? 1 : 0; k < (active(L, 2) ? L->n[2] - 1 : 1); k++)
    for (int j = 1; j < L->n[1] - 1; j++)
      for (int i = 1; i < L->n[0] - 1; i++) {
        int64_t p = idx3(L, i, j, k);
        r[p] = b[p] - M_at(H, L, u, i, j, k);
      }
}

/* ------------------------------------------------------------- smoothers -- */

/* omega-Jacobi (Sec. 4.2): u <- u + omega D^{-1} (b - M u), every node from
 * the old iterate. */
static void jacobi_sweep(const ohier *H, const olevel *L, const cplx *b, cplx *u, double omega) {
  cplx *unew = xcalloc((size_t)L->nn, sizeof(cplx));
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = active(L, 2) ? 1 : 0; k < (active(L, 2) ? L->n[2] - 1 : 1); k++)
    for (int j = 1; j < L->n[1] - 1; j++)
      for (int i = 1; i < L->n[0] - 1; i++) {
        int64_t p = idx3(L, i, j, k);
        unew[p] = u[p] + omega * (b[p] - M_at(H, L, u, i, j, k)) / M_diag(H, L, i, j, k);
      }
  memcpy(u, unew, sizeof(cplx) * (size_t)L->nn);
  free(unew);
}

/* red-black SOR ("omega-red-black Jacobi", Sec. 4.2): nodes with i+j+k even
 * (red) first, then odd (black); each node is relaxed in place,
 * u_p <- u_p + omega (b_p - (M u)_p) / M_pp.  Nodes of one colour only couple
 * to the other colour, so the order inside a colour is immaterial. */
static void rb_sweep(const ohier *H, const olevel *L, const cplx *b, cplx *u, double omega) {
  for (int colour = 0; colour < 2; colour++) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = active(L, 2) ? 1 : 0; k < (active(L, 2) ? L->n[2] - 1 : 1); k++)
      for (int j = 1; j < L->n[1] - 1; j++)
        for (int i = 1; i < L->n[0] - 1; i++) {
          if (((i + j + k) & 1) != colour) continue;
          int64_t p = idx3(L, i, j, k);
          u[p] += omega * (b[p] - M_at(H, L, u, i, j, k)) / M_diag(H, L, i, j, k);
        }
  }
}

static void smooth(const ohier *H, const olevel *L, const cplx *b, cplx *u, int nsweeps) {
  for (int s = 0; s < nsweeps; s++) {
    if (H->smoother == 0) jacobi_sweep(H, L, b, u, H->omega);
    else rb_sweep(H, L, b, u, H->omega);
  }
}

/* ------------------------------------------------------ grid transfers -- */

/* full weighting, index space: tensor product of [1 2 1]/4 over the active
 * axes (9-point [1 2 1; 2 4 2; 1 2 1]/16 in 2D, 27-point /64 in 3D). */
static void restrict_fw(const olevel *F, const olevel *C, const cplx *rf, cplx *rc) {
  zero_vec(rc, C->nn);
  int dk = active(C, 2) ? 1 : 0;
#pragma omp parallel for collapse(2) schedule(static)
  for (int kc = active(C, 2) ? 1 : 0; kc < (active(C, 2) ? C->n[2] - 1 : 1); kc++)
    for (int jc = 1; jc < C->n[1] - 1; jc++)
      for (int ic = 1; ic < C->n[0] - 1; ic++) {
        cplx s = 0;
        for (int c = -dk; c <= dk; c++)
          for (int b = -1; b <= 1; b++)
            for (int a = -1; a <= 1; a++) {
              double wgt = (a == 0 ? 0.5 : 0.25) * (b == 0 ? 0.5 : 0.25) *
                           (dk ? (c == 0 ? 0.5 : 0.25) : 1.0);
              s += wgt * rf[idx3(F, 2 * ic + a, 2 * jc + b, 2 * kc + c)];
            }
        rc[idx3(C, ic, jc, kc)] = s;
      }
}

/* bilinear (trilinear) prolongation in index space, added to u on the fine
 * interior: an even fine index sits on a coarse node (weight 1), an odd one
 * halfway between two (weights 1/2, 1/2). */
static void prolong_add(const olevel *F, const olevel *C, const cplx *ec, cplx *uf) {
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = active(F, 2) ? 1 : 0; k < (active(F, 2) ? F->n[2] - 1 : 1); k++)
    for (int j = 1; j < F->n[1] - 1; j++)
      for (int i = 1; i < F->n[0] - 1; i++) {
        int ci[3][2], nc[3];
        double cw[3][2];
        int fi[3] = {i, j, k};
        for (int a = 0; a < 3; a++) {
          if (!active(F, a)) { nc[a] = 1; ci[a][0] = 0; cw[a][0] = 1; continue; }
          if (fi[a] % 2 == 0) { nc[a] = 1; ci[a][0] = fi[a] / 2; cw[a][0] = 1; }
          else { nc[a] = 2; ci[a][0] = (fi[a] - 1) / 2; ci[a][1] = (fi[a] + 1) / 2; cw[a][0] = cw[a][1] = 0.5; }
        }
        cplx e = 0;
        for (int c = 0; c < nc[2]; c++)
          for (int b = 0; b < nc[1]; b++)
            for (int a = 0; a < nc[0]; a++)
              e += cw[0][a] * cw[1][b] * cw[2][c] * ec[idx3(C, ci[0][a], ci[1][b], ci[2][c])];
        uf[idx3(F, i, j, k)] += e;
      }
}

/* --------------------------------------------------- coarsest direct LU -- */

/* dense LU with partial pivoting of M on the interior unknowns of level L,
 * assembled column by column from M applied to unit vectors. */
static void build_coarse_lu(ohier *H, olevel *L) {
  int nu = 0;
  FOR_INTERIOR(L, i, j, k) nu++;
  L->nunk = nu;
  free(L->lu); free(L->piv); free(L->unk);
  L->lu = xcalloc((size_t)nu * nu, sizeof(cplx));
  L->piv = xcalloc((size_t)nu, sizeof(int));
  L->unk = xcalloc((size_t)nu, sizeof(int64_t));
  int t = 0;
  FOR_INTERIOR(L, i, j, k) L->unk[t++] = idx3(L, i, j, k);
  cplx *e = xcalloc((size_t)L->nn, sizeof(cplx));
  cplx *col = xcalloc((size_t)L->nn, sizeof(cplx));
  for (int c = 0; c < nu; c++) {
    zero_vec(e, L->nn);
    e[L->unk[c]] = 1;
    apply_level(H, L, 1, e, col);
    for (int r = 0; r < nu; r++) L->lu[(size_t)r * nu + c] = col[L->unk[r]];
  }
  free(e); free(col);
  cplx *a = L->lu;
  for (int kk = 0; kk < nu; kk++) {
    int pr = kk;
    double best = cabs(a[(size_t)kk * nu + kk]);
    for (int r = kk + 1; r < nu; r++)
      if (cabs(a[(size_t)r * nu + kk]) > best) { best = cabs(a[(size_t)r * nu + kk]); pr = r; }
    L->piv[kk] = pr;
    if (pr != kk)
      for (int c = 0; c < nu; c++) {
        cplx tmp = a[(size_t)kk * nu + c]; a[(size_t)kk * nu + c] = a[(size_t)pr * nu + c]; a[(size_t)pr * nu + c] = tmp;
      }
    for (int r = kk + 1; r < nu; r++) {
      a[(size_t)r * nu + kk] /= a[(size_t)kk * nu + kk];
      for (int c = kk + 1; c < nu; c++) a[(size_t)r * nu + c] -= a[(size_t)r * nu + kk] * a[(size_t)kk * nu + c];
    }
  }
}

static void coarse_solve(const olevel *L, const cplx *b, cplx *x) {
  int nu = L->nunk;
  cplx *y = xcalloc((size_t)nu, sizeof(cplx));
  for (int r = 0; r < nu; r++) y[r] = b[L->unk[r]];
  for (int kk = 0; kk < nu; kk++)
    if (L->piv[kk] != kk) { cplx t = y[kk]; y[kk] = y[L->piv[kk]]; y[L->piv[kk]] = t; }
  for (int r = 0; r < nu; r++)
    for (int c = 0; c < r; c++) y[r] -= L->lu[(size_t)r * nu + c] * y[c];
  for (int r = nu - 1; r >= 0; r--) {
    for (int c = r + 1; c < nu; c++) y[r] -= L->lu[(size_t)r * nu + c] * y[c];
    y[r] /= L->lu[(size_t)r * nu + r];
  }
  zero_vec(x, L->nn);
  for (int r = 0; r < nu; r++) x[L->unk[r]] = y[r];
  free(y);
}

/* ------------------------------------------------------------ hierarchy -- */

static void free_level(olevel *L) {
  for (int a = 0; a < 3; a++) {
    free(L->z[a]); free(L->am[a]); free(L->ap[a]); free(L->w[a]); free(L->mm[a]); free(L->mp[a]);
  }
  free(L->k2); free(L->b); free(L->u); free(L->r); free(L->lu); free(L->piv); free(L->unk);
  memset(L, 0, sizeof(*L));
}

void ora_destroy(ohier *H) {
  if (!H) return;
  for (int l = 0; l < H->nlev; l++) free_level(&H->lev[l]);
  free(H);
}

/* Fill the preconditioner weights of every level for the selected operator
 * (Sec. 5): CSG rediscretises on the rotated grid z e^{i theta_alpha}; every
 * other kind keeps the original grid. */
static void set_precond_weights(ohier *H) {
  for (int l = 0; l < H->nlev; l++) {
    olevel *L = &H->lev[l];
    for (int a = 0; a < 3; a++) {
      int n = L->n[a];
      if (H->kind == 3) {
        cplx *zr = xcalloc((size_t)n, sizeof(cplx));
        for (int i = 0; i < n; i++) zr[i] = L->z[a][i] * cexp(I * H->p1);
        second_diff_weights(n, zr, L->mm[a], L->mp[a], NULL);
        free(zr);
      } else {
        second_diff_weights(n, L->z[a], L->mm[a], L->mp[a], NULL);
      }
    }
  }
}

/*
 * Build the grid hierarchy (Sec. 3, Sec. 4.2 "rediscretization on the coarse
 * grids").  z per axis comes in from ora_zmap on the finest grid; level l+1
 * keeps every other node of level l, k^2 is injected, the coefficients are
 * recomputed from the coarse z.  nlev levels are built (the caller checks
 * that every active axis has (n-1) divisible by 2^(nlev-1)).
 */
ohier *ora_create(int dim, const int n[3], const double *z0, const double *z1, const double *z2,
                  const double *k2, int nlev) {
  if (nlev < 1 || nlev > ORA_MAXLEV) return NULL;
  ohier *H = xcalloc(1, sizeof(ohier));
  H->dim = dim;
  H->nlev = nlev;
  const double *zin[3] = {z0, z1, z2};
  for (int l = 0; l < nlev; l++) {
    olevel *L = &H->lev[l];
    for (int a = 0; a < 3; a++) {
      if (a >= dim) { L->n[a] = 1; }
      else if (l == 0) { L->n[a] = n[a]; }
      else { L->n[a] = (H->lev[l - 1].n[a] - 1) / 2 + 1; }
    }
    L->nn = (int64_t)L->n[0] * L->n[1] * L->n[2];
    for (int a = 0; a < 3; a++) {
      int na = L->n[a];
      L->z[a] = xcalloc((size_t)na, sizeof(cplx));
      L->am[a] = xcalloc((size_t)na, sizeof(cplx));
      L->ap[a] = xcalloc((size_t)na, sizeof(cplx));
      L->w[a] = xcalloc((size_t)na, sizeof(cplx));
      L->mm[a] = xcalloc((size_t)na, sizeof(cplx));
      L->mp[a] = xcalloc((size_t)na, sizeof(cplx));
      for (int i = 0; i < na; i++) {
        if (a >= dim) L->z[a][i] = 0;
        else if (l == 0) L->z[a][i] = zin[a][2 * i] + I * zin[a][2 * i + 1];
        else L->z[a][i] = H->lev[l - 1].z[a][2 * i];
      }
      second_diff_weights(na, L->z[a], L->am[a], L->ap[a], L->w[a]);
    }
    L->k2 = xcalloc((size_t)L->nn, sizeof(double));
    if (l == 0) memcpy(L->k2, k2, sizeof(double) * (size_t)L->nn);
    else {
      olevel *F = &H->lev[l - 1];
      for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
          for (int i = 0; i < L->n[0]; i++)
            L->k2[idx3(L, i, j, k)] = F->k2[idx3(F, 2 * i, 2 * j, active(L, 2) ? 2 * k : 0)];
    }
    L->b = xcalloc((size_t)L->nn, sizeof(cplx));
    L->u = xcalloc((size_t)L->nn, sizeof(cplx));
    L->r = xcalloc((size_t)L->nn, sizeof(cplx));
  }
  /* default: M = A, V(1,1) RB-GS */
  H->alpha = 1; H->beta = -1; H->c = 0; H->kind = 0;
  H->smoother = 1; H->omega = 1.0; H->nu1 = 1; H->nu2 = 1; H->gf = 1; H->gc = 1;
  set_precond_weights(H);
  build_coarse_lu(H, &H->lev[nlev - 1]);
  return H;
}

/*
 * Select the preconditioner operator (Sec. 5):
 *   kind 0: M = Z = -Lap - k^2                       (alpha, beta, c) = (1, -1, 0)
 *   kind 1: Laplace  M = -Lap                        (1, 0, 0)
 *   kind 2: CSL      M = -Lap + (p1 + i p2) k^2      (1, p1 + i p2, 0)
 *   kind 3: CSG      M = Z on the grid rotated by e^{i p1}
 *   kind 4: QD       M = (1 - i) I + Z / |Re lambda0|, |Re lambda0| = |p1|,
 *                    or max k^2 over the fine grid when p1 = 0 (Sec. 5: the
 *                    largest wavenumber as a rough approximation of lambda0)
 * Returns the |Re lambda0| actually used for QD (0 otherwise).
 */
double ora_set_operator(ohier *H, int kind, double p1, double p2) {
  H->kind = kind; H->p1 = p1; H->p2 = p2;
  double lam = 0;
  switch (kind) {
    case 0: H->alpha = 1; H->beta = -1; H->c = 0; break;
    case 1: H->alpha = 1; H->beta = 0; H->c = 0; break;
    case 2: H->alpha = 1; H->beta = p1 + I * p2; H->c = 0; break;
    case 3: H->alpha = 1; H->beta = -1; H->c = 0; break;
    case 4: {
      lam = fabs(p1); /* Sec. 5 quotes Re(lambda0) as a negative number */
      if (lam == 0) {
        olevel *F = &H->lev[0];
        lam = 0;
        for (int64_t p = 0; p < F->nn; p++) if (F->k2[p] > lam) lam = F->k2[p];
      }
      H->alpha = 1.0 / lam; H->beta = -1.0 / lam; H->c = 1.0 - I;
      H->p1 = lam;
      break;
    }
    default: return -1;
  }
  set_precond_weights(H);
  build_coarse_lu(H, &H->lev[H->nlev - 1]);
  return lam;
}

void ora_set_cycle(ohier *H, int smoother, double omega, int nu1, int nu2, int gf, int gc) {
  H->smoother = smoother; H->omega = omega; H->nu1 = nu1; H->nu2 = nu2; H->gf = gf; H->gc = gc;
}

/* ------------------------------------------------------ Algorithm 1 (MG) -- */

/*
 * u <- MG(l, M_l, b, u, nu1, nu2, C, gf, gc) (Sec. 4.2, Algorithm 1), with
 * the two misprints of the printed algorithm read as: the boxed exact solve
 * applies when l+1 is the coarsest level, and post-smoothing starts from the
 * corrected iterate u^{m+2/3}.  The defect equation on level l+1 is
 * approximated from a zero start by gc recursive calls, the first with
 * indices (gf, gc), the others with (gc, gf).
 */
static void mg(ohier *H, int l, const cplx *b, cplx *u, int gf, int gc) {
  olevel *L = &H->lev[l];
  H->visits[l]++;
  int C = H->nlev - 1;
  if (l == C) { coarse_solve(L, b, u); return; }
  smooth(H, L, b, u, H->nu1);
  olevel *Lc = &H->lev[l + 1];
  residual_level(H, L, b, u, L->r);
  restrict_fw(L, Lc, L->r, Lc->b);
  zero_vec(Lc->u, Lc->nn);
  if (l + 1 == C) {
    H->visits[l + 1]++;
    coarse_solve(Lc, Lc->b, Lc->u);
  } else {
    for (int i = 1; i <= gc; i++) {
      if (i == 1) mg(H, l + 1, Lc->b, Lc->u, gf, gc);
      else mg(H, l + 1, Lc->b, Lc->u, gc, gf);
    }
  }
  prolong_add(L, Lc, Lc->u, u);
  smooth(H, L, b, u, H->nu2);
}

/* one preconditioner application: z = MG(0, M_0, v, 0, ...) from zero */
void ora_mg_apply(ohier *H, const cplx *v, cplx *z) {
  olevel *L = &H->lev[0];
  cplx *bb = xcalloc((size_t)L->nn, sizeof(cplx));
  FOR_INTERIOR(L, i, j, k) { int64_t p = idx3(L, i, j, k); bb[p] = v[p]; }
  zero_vec(z, L->nn);
  H->cycles++;
  if (H->nlev == 1) { H->visits[0]++; coarse_solve(L, bb, z); }
  else mg(H, 0, bb, z, H->gf, H->gc);
  free(bb);
}

/* one cycle of Algorithm 1 from a given iterate u (in/out), b given */
void ora_mg_cycle(ohier *H, const cplx *b, cplx *u) {
  H->cycles++;
  if (H->nlev == 1) { H->visits[0]++; coarse_solve(&H->lev[0], b, u); return; }
  mg(H, 0, b, u, H->gf, H->gc);
}

void ora_get_visits(const ohier *H, int64_t *out) {
  for (int l = 0; l < H->nlev; l++) out[l] = H->visits[l];
}
void ora_reset_visits(ohier *H) {
  memset(H->visits, 0, sizeof(H->visits));
  H->cycles = 0;
}

/* ----------------------------------------------- per-step entry points -- */

void ora_apply(ohier *H, int level, int which, const cplx *x, cplx *y) {
  apply_level(H, &H->lev[level], which, x, y);
}
void ora_residual(ohier *H, int level, const cplx *b, const cplx *u, cplx *r) {
  residual_level(H, &H->lev[level], b, u, r);
}
void ora_smooth(ohier *H, int level, int smoother, double omega, int nsweeps, const cplx *b, cplx *u) {
  int s0 = H->smoother; double w0 = H->omega;
  H->smoother = smoother; H->omega = omega;
  smooth(H, &H->lev[level], b, u, nsweeps);
  H->smoother = s0; H->omega = w0;
}
void ora_restrict(ohier *H, int level_fine, const cplx *rf, cplx *rc) {
  restrict_fw(&H->lev[level_fine], &H->lev[level_fine + 1], rf, rc);
}
void ora_prolong_add(ohier *H, int level_fine, const cplx *ec, cplx *uf) {
  prolong_add(&H->lev[level_fine], &H->lev[level_fine + 1], ec, uf);
}
void ora_coarse_solve(ohier *H, const cplx *b, cplx *x) {
  coarse_solve(&H->lev[H->nlev - 1], b, x);
}
int ora_level_nodes(const ohier *H, int level, int *n_out) {
  if (level < 0 || level >= H->nlev) return -1;
  for (int a = 0; a < 3; a++) n_out[a] = H->lev[level].n[a];
  return 0;
}
/* 1D weights of level l along axis a, for tests (original grid) */
void ora_weights(const ohier *H, int level, int axis, double *am, double *ap, double *w) {
  const olevel *L = &H->lev[level];
  for (int i = 0; i < L->n[axis]; i++) {
    am[2 * i] = creal(L->am[axis][i]); am[2 * i + 1] = cimag(L->am[axis][i]);
    ap[2 * i] = creal(L->ap[axis][i]); ap[2 * i + 1] = cimag(L->ap[axis][i]);
    w[2 * i] = creal(L->w[axis][i]); w[2 * i + 1] = cimag(L->w[axis][i]);
  }
}
void ora_get_k2(const ohier *H, int level, double *out) {
  memcpy(out, H->lev[level].k2, sizeof(double) * (size_t)H->lev[level].nn);
}

/* ------------------------------------------------------------ Krylov -- */

static cplx dotc(const cplx *x, const cplx *y, int64_t n) {
  double sr = 0, si = 0;
#pragma omp parallel for reduction(+ : sr, si) schedule(static)
  for (int64_t p = 0; p < n; p++) {
    cplx t = conj(x[p]) * y[p];
    sr += creal(t); si += cimag(t);
  }
  return sr + I * si;
}
static double nrm2(const cplx *x, int64_t n) { return sqrt(creal(dotc(x, x, n))); }

typedef struct {
  int iterations;     /* Krylov iterations (GMRES: Arnoldi steps; BiCGStab: iterations) */
  int restarts;
  int64_t precond_applications;
  double rel_residual;/* true relative residual ||b - A x|| / ||b|| at exit          */
  int status;         /* 0 converged, 1 not converged, -4 breakdown/NaN               */
} ora_stats;

/* the fine-level operator: which = 0 uses A, 2 uses A^T */
static void opA(ohier *H, int which, const cplx *x, cplx *y) { apply_level(H, &H->lev[0], which, x, y); }

/* right preconditioner for the chosen operator: MG for A; for A^T the
 * transposed problem is preconditioned by W M^{-1} W^{-1} (W = dual widths),
 * which approximates (M^T)^{-1}; the iterate it produces solves A^T y = g
 * because the operator applied is the explicit transpose. */
static void precond(ohier *H, int use_mg, int which, const cplx *v, cplx *z) {
  olevel *L = &H->lev[0];
  if (!use_mg) { memcpy(z, v, sizeof(cplx) * (size_t)L->nn); return; }
  if (which == 0) { ora_mg_apply(H, v, z); return; }
  cplx *t = xcalloc((size_t)L->nn, sizeof(cplx));
  FOR_INTERIOR(L, i, j, k) {
    int64_t p = idx3(L, i, j, k);
    cplx wp = L->w[0][i] * L->w[1][j] * L->w[2][k];
    t[p] = v[p] / wp;
  }
  ora_mg_apply(H, t, z);
  FOR_INTERIOR(L, i, j, k) {
    int64_t p = idx3(L, i, j, k);
    z[p] *= L->w[0][i] * L->w[1][j] * L->w[2][k];
  }
  free(t);
}

static void apply_givens(cplx *cs, cplx *sn, cplx *h, int j) {
  /* rotations G_i = [c s; -conj(s) c] with real c stored as complex */
  for (int i = 0; i < j; i++) {
    cplx t = conj(cs[i]) * h[i] + sn[i] * h[i + 1];
    h[i + 1] = -conj(sn[i]) * h[i] + cs[i] * h[i + 1];
    h[i] = t;
  }
}

static void make_givens(cplx a, cplx b, cplx *c, cplx *s) {
  double na = cabs(a), nb = cabs(b);
  if (nb == 0) { *c = 1; *s = 0; return; }
  if (na == 0) { *c = 0; *s = 1; return; }
  double r = sqrt(na * na + nb * nb);
  cplx ph = a / na;
  *c = na / r;
  *s = ph * conj(b) / r;
}

/*
 * Right-preconditioned restarted GMRES(m) (flexible = 0: x = x0 + M^{-1} V y)
 * or FGMRES(m) (flexible = 1: x = x0 + Z y, z_j = M^{-1} v_j), Arnoldi by
 * modified Gram-Schmidt with the Hermitian inner product, Givens least
 * squares; stops when the true relative residual ||b - A x||/||b|| <= rtol.
 */
static int gmres(ohier *H, int which, int use_mg, int flexible, int m, double rtol, int maxit,
                 const cplx *b_in, cplx *x, ora_stats *st) {
  olevel *L = &H->lev[0];
  int64_t n = L->nn;
  cplx *b = xcalloc((size_t)n, sizeof(cplx));
  FOR_INTERIOR(L, i, j, k) { int64_t p = idx3(L, i, j, k); b[p] = b_in[p]; }
  cplx *V = xcalloc((size_t)n * (m + 1), sizeof(cplx));
  cplx *Z = flexible ? xcalloc((size_t)n * m, sizeof(cplx)) : NULL;
  cplx *w = xcalloc((size_t)n, sizeof(cplx));
  cplx *t = xcalloc((size_t)n, sizeof(cplx));
  cplx *Hm = xcalloc((size_t)(m + 1) * m, sizeof(cplx));
  cplx *cs = xcalloc((size_t)m, sizeof(cplx)), *sn = xcalloc((size_t)m, sizeof(cplx));
  cplx *g = xcalloc((size_t)m + 1, sizeof(cplx)), *y = xcalloc((size_t)m, sizeof(cplx));
  double bn = nrm2(b, n);
  memset(st, 0, sizeof(*st));
  int status = 1;
  if (bn == 0) { zero_vec(x, n); st->status = 0; status = 0; goto done; }
  for (int64_t p = 0; p < n; p++) if (b[p] != b[p]) { status = -4; goto done; }
  int it = 0;
  for (;;) {
    opA(H, which, x, t);
    for (int64_t p = 0; p < n; p++) V[p] = b[p] - t[p];
    double beta = nrm2(V, n);
    st->rel_residual = beta / bn;
    if (!(beta == beta)) { status = -4; break; }
    if (beta <= rtol * bn) { status = 0; break; }
    if (it >= maxit) { status = 1; break; }
    for (int64_t p = 0; p < n; p++) V[p] /= beta;
    memset(g, 0, sizeof(cplx) * (m + 1));
    g[0] = beta;
    int jlast = 0;
    for (int jj = 0; jj < m && it < maxit; jj++) {
      cplx *vj = V + (size_t)jj * n;
      cplx *zj = flexible ? Z + (size_t)jj * n : t;
      precond(H, use_mg, which, vj, zj);
      st->precond_applications++;
      opA(H, which, zj, w);
      cplx *h = Hm + (size_t)jj * (m + 1);
      for (int i = 0; i <= jj; i++) {
        cplx *vi = V + (size_t)i * n;
        h[i] = dotc(vi, w, n);
        for (int64_t p = 0; p < n; p++) w[p] -= h[i] * vi[p];
      }
      double hn = nrm2(w, n);
      h[jj + 1] = hn;
      it++;
      jlast = jj + 1;
      if (hn > 0) {
        cplx *vn = V + (size_t)(jj + 1) * n;
        for (int64_t p = 0; p < n; p++) vn[p] = w[p] / hn;
      }
      apply_givens(cs, sn, h, jj);
      make_givens(h[jj], h[jj + 1], &cs[jj], &sn[jj]);
      cplx hj = conj(cs[jj]) * h[jj] + sn[jj] * h[jj + 1];
      h[jj] = hj; h[jj + 1] = 0;
      cplx gj = conj(cs[jj]) * g[jj];
      g[jj + 1] = -conj(sn[jj]) * g[jj];
      g[jj] = gj;
      if (cabs(g[jj + 1]) <= rtol * bn || hn == 0) break;
    }
    /* back substitution R y = g */
    for (int r = jlast - 1; r >= 0; r--) {
      cplx s = g[r];
      for (int c = r + 1; c < jlast; c++) s -= Hm[(size_t)c * (m + 1) + r] * y[c];
      y[r] = s / Hm[(size_t)r * (m + 1) + r];
    }
    if (flexible) {
      for (int c = 0; c < jlast; c++)
        for (int64_t p = 0; p < n; p++) x[p] += y[c] * Z[(size_t)c * n + p];
    } else {
      zero_vec(w, n);
      for (int c = 0; c < jlast; c++)
        for (int64_t p = 0; p < n; p++) w[p] += y[c] * V[(size_t)c * n + p];
      precond(H, use_mg, which, w, t);
      st->precond_applications++;
      for (int64_t p = 0; p < n; p++) x[p] += t[p];
    }
    st->restarts++;
  }
  st->iterations = it;
done:
  st->status = status;
  free(b); free(V); free(Z); free(w); free(t); free(Hm); free(cs); free(sn); free(g); free(y);
  return status;
}

/*
 * Right-preconditioned Bi-CGSTAB (van der Vorst), shadow residual r^ = r0,
 * Hermitian inner products; two preconditioner applications and two operator
 * applications per iteration (Sec. 5).  The recursive residual drives the
 * iteration; when it passes rtol the true residual is recomputed and the
 * method restarts from the current iterate if the true residual has not.
 */
static int bicgstab(ohier *H, int which, int use_mg, double rtol, int maxit,
                    const cplx *b_in, cplx *x, ora_stats *st) {
  olevel *L = &H->lev[0];
  int64_t n = L->nn;
  cplx *b = xcalloc((size_t)n, sizeof(cplx));
  FOR_INTERIOR(L, i, j, k) { int64_t p = idx3(L, i, j, k); b[p] = b_in[p]; }
  cplx *r = xcalloc((size_t)n, sizeof(cplx)), *rh = xcalloc((size_t)n, sizeof(cplx));
  cplx *p_ = xcalloc((size_t)n, sizeof(cplx)), *v = xcalloc((size_t)n, sizeof(cplx));
  cplx *ph = xcalloc((size_t)n, sizeof(cplx)), *s = xcalloc((size_t)n, sizeof(cplx));
  cplx *sh = xcalloc((size_t)n, sizeof(cplx)), *t = xcalloc((size_t)n, sizeof(cplx));
  double bn = nrm2(b, n);
  memset(st, 0, sizeof(*st));
  int status = 1, it = 0;
  if (bn == 0) { zero_vec(x, n); status = 0; goto done; }
  for (int64_t q = 0; q < n; q++) if (b[q] != b[q]) { status = -4; goto done; }
  for (;;) {
    opA(H, which, x, t);
    for (int64_t q = 0; q < n; q++) r[q] = b[q] - t[q];
    double rn = nrm2(r, n);
    st->rel_residual = rn / bn;
    if (!(rn == rn)) { status = -4; break; }
    if (rn <= rtol * bn) { status = 0; break; }
    if (it >= maxit) { status = 1; break; }
    memcpy(rh, r, sizeof(cplx) * (size_t)n);
    cplx rho = 1, alpha = 1, omega = 1;
    zero_vec(v, n); zero_vec(p_, n);
    int inner_done = 0;
    while (it < maxit && !inner_done) {
      cplx rho1 = dotc(rh, r, n);
      if (rho1 == 0) { status = -4; goto out; }
      cplx beta = (rho1 / rho) * (alpha / omega);
      rho = rho1;
      for (int64_t q = 0; q < n; q++) p_[q] = r[q] + beta * (p_[q] - omega * v[q]);
      precond(H, use_mg, which, p_, ph);
      st->precond_applications++;
      opA(H, which, ph, v);
      cplx rv = dotc(rh, v, n);
      if (rv == 0) { status = -4; goto out; }
      alpha = rho / rv;
      for (int64_t q = 0; q < n; q++) s[q] = r[q] - alpha * v[q];
      it++;
      if (nrm2(s, n) <= rtol * bn) {
        for (int64_t q = 0; q < n; q++) x[q] += alpha * ph[q];
        inner_done = 1;
        break;
      }
      precond(H, use_mg, which, s, sh);
      st->precond_applications++;
      opA(H, which, sh, t);
      double tt = creal(dotc(t, t, n));
      if (tt == 0) { status = -4; goto out; }
      omega = dotc(t, s, n) / tt;
      for (int64_t q = 0; q < n; q++) {
        x[q] += alpha * ph[q] + omega * sh[q];
        r[q] = s[q] - omega * t[q];
      }
      double rn2 = nrm2(r, n);
      if (!(rn2 == rn2)) { status = -4; goto out; }
      if (rn2 <= rtol * bn) inner_done = 1;
      if (omega == 0) { status = -4; goto out; }
    }
    st->restarts++;
  }
out:
  if (status == -4) {
    opA(H, which, x, t);
    for (int64_t q = 0; q < n; q++) r[q] = b[q] - t[q];
    st->rel_residual = nrm2(r, n) / bn;
  }
  st->iterations = it;
done:
  st->status = status;
  free(b); free(r); free(rh); free(p_); free(v); free(ph); free(s); free(sh); free(t);
  return status;
}

/*
 * Solve A x = b (which = 0) or A^T x = b (which = 2) on the finest grid.
 * krylov: 0 GMRES(m), 1 FGMRES(m), 2 Bi-CGSTAB.  use_mg = 0 runs the Krylov
 * method unpreconditioned.  x holds the initial guess on entry.
 * stats_out: {iterations, restarts, precond_applications, rel_residual, status}.
 */
int ora_solve(ohier *H, int which, int krylov, int use_mg, int m, double rtol, int maxit,
              const cplx *b, cplx *x, double *stats_out) {
  ora_stats st;
  int rc;
  if (krylov == 2) rc = bicgstab(H, which, use_mg, rtol, maxit, b, x, &st);
  else rc = gmres(H, which, use_mg, krylov == 1, m, rtol, maxit, b, x, &st);
  stats_out[0] = st.iterations;
  stats_out[1] = st.restarts;
  stats_out[2] = (double)st.precond_applications;
  stats_out[3] = st.rel_residual;
  stats_out[4] = st.status;
  return rc;
}

int ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* threads of the parallel loops from now on (timing only; the reductions'
 * summation order, and so their last bits, depends on the count) */
void ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
