/*
 * slmpp_oracle.c -- plain FP64 CPU oracle for the SL-MPP5/7 Vlasov sweeps.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the HIP library: every formula below is written out again from the
 * paper (Tanaka, Yoshikawa, Minoshima & Yoshida, "Multidimensional
 * Vlasov-Poisson Simulations with High-order Monotonicity- and
 * Positivity-preserving Schemes", arXiv:1702.08521).
 *
 * It is deliberately slow and literal: one pencil at a time, the interface
 * flux built in the order the paper gives it (CSL polynomial -> MP
 * constraint -> PP limiter -> conservative update), every intermediate in
 * double precision, no blocking or fusion.  Pencils are independent, so an
 * OpenMP loop over pencils changes nothing in the arithmetic.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math).
 *
 * Readings of points the paper leaves open (each one is also listed in the
 * design notes of the repository):
 *   R1  Large CFL.  The departure point splits as xi = N + zeta with
 *       N = floor(xi + 1/2), so zeta lies in [-1/2, 1/2).  Cell i of the
 *       new pencil takes the CSL update of the extended old pencil shifted
 *       by N cells (the CSL identity of Sec. 2.1.2 applied to the foot of
 *       the characteristic, which is cell i-N moved by zeta).
 *   R2  Negative speed.  The paper treats c > 0 only (Sec. 2.1); for
 *       zeta < 0 the shifted pencil is reversed, advanced with |zeta| and
 *       reversed back.
 *   R3  PP denominators.  theta = U^UP / (U^UP - U) is used only when the
 *       denominator is positive; otherwise theta = 0.  theta is clamped
 *       to [0, 1] (the paper requires 0 <= theta <= 1).
 *   R4  median(a, b, c) is the middle value of the three numbers.
 *   R5  Boundaries.  Periodic axes wrap; outflow axes read zero outside
 *       the domain, so nothing flows in.
 *   R6  Green function at k = 0 is zero (mean density removed), and with
 *       unequal mesh spacings the one-dimensional symbols are summed with
 *       their own 1/Delta_l^2 (reduces to the printed form for equal
 *       spacings).
 *   R7  Four-point FDA: the printed difference has the opposite sign of
 *       the derivative; the derivative itself is used here.
 *   R9  Isolated boundaries (Sec. 2.2, doubling-up method).  The real-
 *       space Green function is g(r) = -kappa / (4 pi r) (the attractive
 *       sign for kappa = 4 pi G), sampled at cell-centre separations on the
 *       grid doubled along each axis with minimum-image distances; at r = 0
 *       it takes the mean of -kappa / (4 pi r) over one cell.  The forces
 *       use the FDA on the doubled grid, whose potential beyond the
 *       physical cells is the isolated potential there.  D = 3 only.
 *   R8  RK-MP(P)5/7 (Sec. 2.1.1).  Each TVD-RK stage recomputes the
 *       interface values from the stage data extended by the boundary
 *       condition (as R5); c < 0 reverses the pencil as in R2.  The PP
 *       limiter is the Sec. 2.1.1 one with the CFL number nu of the step.
 *       |nu| <= 1 is required (no integer shift exists in this scheme).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_BC_PERIODIC 0
#define ORACLE_BC_OUTFLOW 1

#define ORACLE_LIM_NONE 0 /* CSL flux only (no constraint)          */
#define ORACLE_LIM_MP 1   /* SL-MP: CSL + MP constraint             */
#define ORACLE_LIM_MPP 2  /* SL-MPP: CSL + MP constraint + PP limiter */

/* Phase-space grid.  Array layout: f[x1..xD][v1..vD], last axis fastest. */
typedef struct {
  int32_t D;
  int32_t order;      /* 5 or 7 */
  int32_t limiter;    /* ORACLE_LIM_* */
  int32_t poisson_order; /* 2, 4 or 6 */
  int64_t nx[3], nv[3];
  double x_lo[3], x_hi[3], v_lo[3], v_hi[3];
  double alpha;       /* MP parameter (App. A uses 4) */
  double kappa;       /* Poisson coupling: lap(phi) = kappa * rho */
  int32_t x_bc, v_bc;
  int32_t time_scheme; /* ORACLE_TIME_SL or ORACLE_TIME_RK3 */
  int32_t merge_kicks; /* 1: oracle_steps merges consecutive velocity half-steps */
  int32_t isolated;    /* 1: isolated-boundary field solve (D = 3) */
  int32_t pad;
} oracle_grid;

#define ORACLE_TIME_SL 0  /* semi-Lagrangian update, Eq. (SL)          */
#define ORACLE_TIME_RK3 1 /* method of lines + three-stage TVD-RK, Eq. (RK) */

/* ------------------------------------------------------------------ */
/* Scalar pieces of the interface flux                                 */
/* ------------------------------------------------------------------ */

/* minmod of two numbers: the one of smaller magnitude when both have the
 * same sign, otherwise zero (App. A, steps 2 and 4). */
double oracle_minmod2(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

double oracle_minmod4(double a, double b, double c, double d) {
  if (a > 0.0 && b > 0.0 && c > 0.0 && d > 0.0) {
    double m = a;
    if (b < m) m = b;
    if (c < m) m = c;
    if (d < m) m = d;
    return m;
  }
  if (a < 0.0 && b < 0.0 && c < 0.0 && d < 0.0) {
    double m = a;
    if (b > m) m = b;
    if (c > m) m = c;
    if (d > m) m = d;
    return m;
  }
  return 0.0;
}

static double min3(double a, double b, double c) {
  double m = a < b ? a : b;
  return m < c ? m : c;
}
static double max3(double a, double b, double c) {
  double m = a > b ? a : b;
  return m > c ? m : c;
}

/* Middle value of three numbers (reading R4). */
double oracle_median3(double a, double b, double c) {
  double lo = a < b ? a : b;
  double hi = a < b ? b : a;
  if (c <= lo) return lo;
  if (c >= hi) return hi;
  return c;
}

/* MP constraint of App. A for the interface downwind of cell "0":
 *   fm2 = f_{i-2}, fm1 = f_{i-1}, f0 = f_i (upwind cell), fp1 = f_{i+1},
 *   fp2 = f_{i+2}, fint = unconstrained interface value.
 * The seven steps are followed in order, including the early accept. */
double oracle_mp(double fint, double fm2, double fm1, double f0, double fp1,
                 double fp2, double alpha) {
  /* step 2 */
  double fstar = f0 + oracle_minmod2(fp1 - f0, alpha * (f0 - fm1));
  /* step 3 */
  if ((fint - f0) * (fint - fstar) < 0.0) return fint;
  /* step 4: curvatures d_j = f_{j-1} + f_{j+1} - 2 f_j */
  double dm1 = fm2 + f0 - 2.0 * fm1;
  double d0 = fm1 + fp1 - 2.0 * f0;
  double dp1 = f0 + fp2 - 2.0 * fp1;
  double dM4_plus = oracle_minmod4(4.0 * d0 - dp1, 4.0 * dp1 - d0, d0, dp1);
  double dM4_minus = oracle_minmod4(4.0 * dm1 - d0, 4.0 * d0 - dm1, dm1, d0);
  /* step 5 */
  double fUL = f0 + alpha * (f0 - fm1);
  double fAV = (f0 + fp1) / 2.0;
  double fMD = fAV - dM4_plus / 2.0;
  double fLC = f0 + (f0 - fm1) / 2.0 + 4.0 * dM4_minus / 3.0;
  /* step 6 */
  double lo_a = min3(f0, fp1, fMD), lo_b = min3(f0, fUL, fLC);
  double hi_a = max3(f0, fp1, fMD), hi_b = max3(f0, fUL, fLC);
  double f_min = lo_a > lo_b ? lo_a : lo_b;
  double f_max = hi_a < hi_b ? hi_a : hi_b;
  /* step 7 */
  return oracle_median3(fint, f_min, f_max);
}

/* theta for one side of the PP limiter (Sec. 2.1.1, reading R3). */
static double pp_theta(double u_up, double u) {
  if (!(u < 0.0)) return 1.0;
  double den = u_up - u;
  if (!(den > 0.0)) return 0.0;
  double t = u_up / den;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  return t;
}

/* PP limiter of Sec. 2.1.1 for the interface between the upwind cell fl
 * (f_i) and the downwind cell fr (f_{i+1}); nu is the (fractional) CFL
 * number of the update.  The upwind interface value is f_i. */
double oracle_pp(double phibar, double fl, double fr, double nu) {
  double u_plus = fl - 2.0 * nu * phibar;     /* U_i^+           */
  double u_minus = fr + 2.0 * nu * phibar;    /* U_{i+1}^-       */
  double u_up_plus = fl - 2.0 * nu * fl;      /* U_i^{UP,+}      */
  double u_up_minus = fr + 2.0 * nu * fl;     /* U_{i+1}^{UP,-}  */
  double th_plus = pp_theta(u_up_plus, u_plus);
  double th_minus = pp_theta(u_up_minus, u_minus);
  double th = th_plus < th_minus ? th_plus : th_minus;
  return th * phibar + (1.0 - th) * fl;
}

/* CSL flux Phi_{i-1/2} = sum_j C_j zeta^j (fifth order, s = f_{i-3..i+1})
 * or sum_j D_j zeta^j (seventh order, s = f_{i-4..i+2}), Sec. 2.1.2.
 * The coefficient rows are the printed ones. */
double oracle_csl_flux(const double* s, int order, double zeta) {
  if (order == 5) {
    const double fm3 = s[0], fm2 = s[1], fm1 = s[2], f0 = s[3], fp1 = s[4];
    double C0 = fm3 / 30.0 - 13.0 / 60.0 * fm2 + 47.0 / 60.0 * fm1 +
                9.0 / 20.0 * f0 - fp1 / 20.0;
    double C1 = -fm2 / 24.0 + 5.0 / 8.0 * fm1 - 5.0 / 8.0 * f0 + fp1 / 24.0;
    double C2 = -fm3 / 24.0 + fm2 / 4.0 - fm1 / 3.0 + f0 / 12.0 + fp1 / 24.0;
    double C3 = fm2 / 24.0 - fm1 / 8.0 + f0 / 8.0 - fp1 / 24.0;
    double C4 = fm3 / 120.0 - fm2 / 30.0 + fm1 / 20.0 - f0 / 30.0 + fp1 / 120.0;
    return C0 + zeta * (C1 + zeta * (C2 + zeta * (C3 + zeta * C4)));
  } else {
    const double fm4 = s[0], fm3 = s[1], fm2 = s[2], fm1 = s[3], f0 = s[4],
                 fp1 = s[5], fp2 = s[6];
    double D0 = -fm4 / 140.0 + 5.0 / 84.0 * fm3 - 101.0 / 420.0 * fm2 +
                319.0 / 420.0 * fm1 + 107.0 / 210.0 * f0 - 19.0 / 210.0 * fp1 +
                fp2 / 105.0;
    double D1 = fm3 / 180.0 - 5.0 / 72.0 * fm2 + 49.0 / 72.0 * fm1 -
                49.0 / 72.0 * f0 + 5.0 / 72.0 * fp1 - fp2 / 180.0;
    double D2 = 7.0 / 720.0 * fm4 - 19.0 / 240.0 * fm3 + 7.0 / 24.0 * fm2 -
                23.0 / 72.0 * fm1 + f0 / 48.0 + 7.0 / 80.0 * fp1 - fp2 / 90.0;
    double D3 = -fm3 / 144.0 + 11.0 / 144.0 * fm2 - 7.0 / 36.0 * fm1 +
                7.0 / 36.0 * f0 - 11.0 / 144.0 * fp1 + fp2 / 144.0;
    double D4 = -fm4 / 360.0 + fm3 / 48.0 - 13.0 / 240.0 * fm2 +
                23.0 / 360.0 * fm1 - f0 / 30.0 + fp1 / 240.0 + fp2 / 720.0;
    double D5 = fm3 / 720.0 - fm2 / 144.0 + fm1 / 72.0 - f0 / 72.0 +
                fp1 / 144.0 - fp2 / 720.0;
    double D6 = fm4 / 5040.0 - fm3 / 840.0 + fm2 / 336.0 - fm1 / 252.0 +
                f0 / 336.0 - fp1 / 840.0 + fp2 / 5040.0;
    return D0 +
           zeta * (D1 + zeta * (D2 + zeta * (D3 + zeta * (D4 + zeta * (D5 + zeta * D6)))));
  }
}

/* Constrained interface value at the interface m-1/2 of the working pencil
 * r (r[k] for k = m-4 .. m+2 must be addressable), Sec. 2.1.2:
 *   Phi    = CSL polynomial,
 *   Phibar = MP(Phi; r_{m-3}, r_{m-2}, r_{m-1}, r_m, r_{m+1}),
 *   Phihat = PP(Phibar; r_{m-1}, r_m). */
static double interface_flux(const double* r, int64_t m, int order, int limiter,
                             double alpha, double nu) {
  double phi;
  if (order == 5)
    phi = oracle_csl_flux(r + m - 3, 5, nu);
  else
    phi = oracle_csl_flux(r + m - 4, 7, nu);
  if (limiter >= ORACLE_LIM_MP)
    phi = oracle_mp(phi, r[m - 3], r[m - 2], r[m - 1], r[m], r[m + 1], alpha);
  if (limiter >= ORACLE_LIM_MPP) phi = oracle_pp(phi, r[m - 1], r[m], nu);
  return phi;
}

/* Value of the old pencil g at integer position k, extended beyond the
 * domain by the boundary condition (reading R5). */
static double extended(const double* g, int64_t n, int64_t stride, int64_t k,
                       int bc) {
  if (bc == ORACLE_BC_PERIODIC) {
    k %= n;
    if (k < 0) k += n;
    return g[k * stride];
  }
  if (k < 0 || k >= n) return 0.0;
  return g[k * stride];
}

#define ORACLE_GHOST 5 /* >= stencil half-width + 1 */

/* One SL step of a single pencil g[0], g[stride], ..., g[(n-1)*stride]
 * with departure offset xi = c dt / h (in cells).  `work` needs
 * 2*(n + 2*ORACLE_GHOST) + 1 doubles. */
void oracle_sweep_pencil_work(double* g, int64_t n, int64_t stride, double xi,
                              int order, int limiter, double alpha, int bc,
                              double* work) {
  if (n <= 0) return;
  const double Nd = floor(xi + 0.5); /* reading R1 */
  const int64_t N = (int64_t)Nd;
  const double zeta = xi - Nd;
  const int mirror = zeta < 0.0; /* reading R2 */
  const double nu = mirror ? -zeta : zeta;
  double* r = work + ORACLE_GHOST;            /* r[-GHOST .. n+GHOST) */
  double* F = work + n + 2 * ORACLE_GHOST;    /* F[0 .. n]            */
  /* working pencil: r_m = q_m = g_{m-N}   (no mirror)
   *                 r_m = q_{n-1-m} = g_{n-1-m-N}   (mirror)          */
  for (int64_t m = -ORACLE_GHOST; m < n + ORACLE_GHOST; ++m) {
    int64_t k = mirror ? (n - 1 - m - N) : (m - N);
    r[m] = extended(g, n, stride, k, bc);
  }
  /* interface values Phihat_{m-1/2}, m = 0 .. n */
  for (int64_t m = 0; m <= n; ++m)
    F[m] = interface_flux(r, m, order, limiter, alpha, nu);
  /* conservative update, Eq. (SL) */
  for (int64_t m = 0; m < n; ++m) {
    double out = r[m] - nu * (F[m + 1] - F[m]);
    int64_t i = mirror ? (n - 1 - m) : m;
    g[i * stride] = out;
  }
}

void oracle_sweep_pencil(double* g, int64_t n, int64_t stride, double xi, int order,
                         int limiter, double alpha, int bc) {
  double* work = (double*)malloc(sizeof(double) * (2 * (n + 2 * ORACLE_GHOST) + 1));
  oracle_sweep_pencil_work(g, n, stride, xi, order, limiter, alpha, bc, work);
  free(work);
}

/* Interpolated interface value f^int_{m-1/2} of the MP schemes (the
 * printed fifth- and seventh-order formulas, Sec. 2.1.1), from the working
 * pencil r around the upwind cell m-1. */
static double rk_interp(const double* r, int64_t m, int order) {
  if (order == 5)
    return (2.0 * r[m - 3] - 13.0 * r[m - 2] + 47.0 * r[m - 1] + 27.0 * r[m] -
            3.0 * r[m + 1]) / 60.0;
  return (-3.0 * r[m - 4] + 25.0 * r[m - 3] - 101.0 * r[m - 2] + 319.0 * r[m - 1] +
          214.0 * r[m] - 38.0 * r[m + 1] + 4.0 * r[m + 2]) / 420.0;
}

/* The same interpolation on a stencil s = f_{i-3..i+1} (fifth order) or
 * f_{i-4..i+2} (seventh order): f^int_{i-1/2}. */
double oracle_rk_interp(const double* s, int order) {
  return rk_interp(s + (order == 5 ? 3 : 4), 0, order);
}

/* L_m(u) = fhat_{m+1/2} - fhat_{m-1/2} for m = 0 .. n-1 of the working
 * pencil u (n values, extended by the boundary condition into r), with
 * fbar = MP(f^int) and fhat = PP(fbar; u_{m-1}, u_m) (Sec. 2.1.1). */
static void rk_operator(const double* u, int64_t n, int order, int limiter, double alpha,
                        int bc, double nu, double* r, double* F, double* L) {
  for (int64_t m = -ORACLE_GHOST; m < n + ORACLE_GHOST; ++m)
    r[m] = extended(u, n, 1, m, bc);
  for (int64_t m = 0; m <= n; ++m) {
    double phi = rk_interp(r, m, order);
    if (limiter >= ORACLE_LIM_MP)
      phi = oracle_mp(phi, r[m - 3], r[m - 2], r[m - 1], r[m], r[m + 1], alpha);
    if (limiter >= ORACLE_LIM_MPP) phi = oracle_pp(phi, r[m - 1], r[m], nu);
    F[m] = phi;
  }
  for (int64_t m = 0; m < n; ++m) L[m] = F[m + 1] - F[m];
}

/* One RK-MP(P) step of a single pencil with CFL number nu = c dt / h,
 * Eq. (RK):  f1 = f - nu L(f),  f2 = 3/4 f + 1/4 (f1 - nu L(f1)),
 * f^{n+1} = 1/3 f + 2/3 (f2 - nu L(f2)).  `work` needs
 * ORACLE_RK_WORK(n) doubles.  Returns -1 (and leaves g) when |nu| > 1. */
#define ORACLE_RK_WORK(n) (6 * ((n) + 2 * ORACLE_GHOST) + 1)
int oracle_rk_pencil_work(double* g, int64_t n, int64_t stride, double xi, int order,
                          int limiter, double alpha, int bc, double* work) {
  if (n <= 0) return 0;
  if (!(fabs(xi) <= 1.0)) return -1;
  const int mirror = xi < 0.0; /* reading R8 (as R2) */
  const double nu = mirror ? -xi : xi;
  const int64_t span = n + 2 * ORACLE_GHOST;
  double* u0 = work;               /* f^n in working orientation */
  double* u1 = work + span;        /* stage values               */
  double* L = work + 2 * span;
  double* F = work + 3 * span;
  double* r = work + 4 * span + ORACLE_GHOST;
  for (int64_t m = 0; m < n; ++m) u0[m] = g[(mirror ? (n - 1 - m) : m) * stride];
  /* stage 1 */
  rk_operator(u0, n, order, limiter, alpha, bc, nu, r, F, L);
  for (int64_t m = 0; m < n; ++m) u1[m] = u0[m] - nu * L[m];
  /* stage 2 */
  rk_operator(u1, n, order, limiter, alpha, bc, nu, r, F, L);
  for (int64_t m = 0; m < n; ++m) u1[m] = 0.75 * u0[m] + 0.25 * (u1[m] - nu * L[m]);
  /* stage 3 */
  rk_operator(u1, n, order, limiter, alpha, bc, nu, r, F, L);
  for (int64_t m = 0; m < n; ++m) {
    const double out = u0[m] / 3.0 + 2.0 / 3.0 * (u1[m] - nu * L[m]);
    g[(mirror ? (n - 1 - m) : m) * stride] = out;
  }
  return 0;
}

int oracle_rk_pencil(double* g, int64_t n, int64_t stride, double xi, int order, int limiter,
                     double alpha, int bc) {
  double* work = (double*)malloc(sizeof(double) * ORACLE_RK_WORK(n));
  int rc = oracle_rk_pencil_work(g, n, stride, xi, order, limiter, alpha, bc, work);
  free(work);
  return rc;
}

/* One sweep of a pencil with the time scheme of the grid. */
static int scheme_pencil(const oracle_grid* gr, double* g, int64_t n, int64_t stride, double xi,
                         int bc, double* work) {
  if (gr->time_scheme == ORACLE_TIME_RK3)
    return oracle_rk_pencil_work(g, n, stride, xi, gr->order, gr->limiter, gr->alpha, bc, work);
  oracle_sweep_pencil_work(g, n, stride, xi, gr->order, gr->limiter, gr->alpha, bc, work);
  return 0;
}

/* All pencils of an array viewed as [outer][n][inner], same xi for all. */
void oracle_sweep_lines(double* f, int64_t outer, int64_t n, int64_t inner,
                        double xi, int order, int limiter, double alpha, int bc) {
  const int64_t npen = outer * inner;
#pragma omp parallel
  {
    double* work = (double*)malloc(sizeof(double) * (2 * (n + 2 * ORACLE_GHOST) + 1));
#pragma omp for schedule(static)
    for (int64_t p = 0; p < npen; ++p) {
      int64_t o = p / inner, j = p % inner;
      oracle_sweep_pencil_work(f + o * n * inner + j, n, inner, xi, order, limiter,
                               alpha, bc, work);
    }
    free(work);
  }
}

/* ------------------------------------------------------------------ */
/* Phase-space geometry                                                */
/* ------------------------------------------------------------------ */

static void grid_dims(const oracle_grid* g, int64_t* dims) {
  for (int l = 0; l < g->D; ++l) {
    dims[l] = g->nx[l];
    dims[g->D + l] = g->nv[l];
  }
}

static int64_t prod_range(const int64_t* dims, int a, int b) {
  int64_t p = 1;
  for (int k = a; k < b; ++k) p *= dims[k];
  return p;
}

/* Cell centre lo + (j + 1/2) * (hi - lo) / n, Sec. 2.1 */
double oracle_cell_center(double lo, double hi, int64_t n, int64_t j) {
  double d = (hi - lo) / (double)n;
  return lo + ((double)j + 0.5) * d;
}

/* Departure offset in cells: xi = c dt / h */
double oracle_xi(double c, double dt, double h) { return (c * dt) / h; }

/* Advection along x_dim with speed v_dim, Eq. (adv_pos). */
int oracle_advect_x(const oracle_grid* g, double* f, int dim, double dt) {
  int64_t dims[6];
  grid_dims(g, dims);
  const int nd = 2 * g->D;
  const int a = dim;
  const int64_t outer = prod_range(dims, 0, a);
  const int64_t n = dims[a];
  const int64_t inner = prod_range(dims, a + 1, nd);
  const int64_t vstride = prod_range(dims, g->D + dim + 1, nd); /* stride of v_dim */
  const int64_t nvd = g->nv[dim];
  const double h = (g->x_hi[dim] - g->x_lo[dim]) / (double)g->nx[dim];
  const int64_t npen = outer * inner;
  int bad = 0;
#pragma omp parallel reduction(| : bad)
  {
    double* work = (double*)malloc(sizeof(double) * ORACLE_RK_WORK(n));
#pragma omp for schedule(static)
    for (int64_t p = 0; p < npen; ++p) {
      int64_t o = p / inner, j = p % inner;
      int64_t jv = (j / vstride) % nvd;
      double c = oracle_cell_center(g->v_lo[dim], g->v_hi[dim], nvd, jv);
      double xi = oracle_xi(c, dt, h);
      bad |= scheme_pencil(g, f + o * n * inner + j, n, inner, xi, g->x_bc, work) != 0;
    }
    free(work);
  }
  return bad ? -1 : 0;
}

/* Advection along v_dim with speed accel[dim-th component at x],
 * Eq. (adv_vel).  accel holds prod(nx) values for this component. */
int oracle_advect_v(const oracle_grid* g, double* f, int dim, double dt,
                     const double* accel) {
  int64_t dims[6];
  grid_dims(g, dims);
  const int nd = 2 * g->D;
  const int a = g->D + dim;
  const int64_t outer = prod_range(dims, 0, a);
  const int64_t n = dims[a];
  const int64_t inner = prod_range(dims, a + 1, nd);
  const int64_t vblock = prod_range(dims, g->D, a); /* v axes before v_dim */
  const double h = (g->v_hi[dim] - g->v_lo[dim]) / (double)g->nv[dim];
  const int64_t npen = outer * inner;
  int bad = 0;
#pragma omp parallel reduction(| : bad)
  {
    double* work = (double*)malloc(sizeof(double) * ORACLE_RK_WORK(n));
#pragma omp for schedule(static)
    for (int64_t p = 0; p < npen; ++p) {
      int64_t o = p / inner, j = p % inner;
      int64_t ix = o / vblock;
      double xi = oracle_xi(accel[ix], dt, h);
      bad |= scheme_pencil(g, f + o * n * inner + j, n, inner, xi, g->v_bc, work) != 0;
    }
    free(work);
  }
  return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Velocity moment and field solve                                     */
/* ------------------------------------------------------------------ */

/* Compensated (Neumaier) accumulator. */
typedef struct {
  double s, c;
} ksum_t;
static void ksum_add(ksum_t* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

/* Velocity moments of each spatial cell (Sec. 2.3: density, mean
 * velocities, velocity dispersions):
 *   rho(x)       = dv^D sum_v f,
 *   u_l(x)       = dv^D sum_v f v_l / rho,
 *   sigma2_l(x)  = dv^D sum_v f (v_l - u_l)^2 / rho,
 * with v_l the cell centres; mean and disp hold D * prod(nx) values
 * (component-major).  Cells with rho = 0 get u = sigma2 = 0. */
void oracle_velocity_moments(const oracle_grid* g, const double* f, double* rho, double* mean,
                             double* disp) {
  int64_t nxs = 1, nvs = 1;
  double dvol = 1.0;
  for (int l = 0; l < g->D; ++l) {
    nxs *= g->nx[l];
    nvs *= g->nv[l];
    dvol *= (g->v_hi[l] - g->v_lo[l]) / (double)g->nv[l];
  }
#pragma omp parallel for schedule(static)
  for (int64_t ix = 0; ix < nxs; ++ix) {
    const double* b = f + ix * nvs;
    ksum_t s0 = {0, 0}, s1[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t k = 0; k < nvs; ++k) {
      int64_t rem = k;
      double v[3] = {0, 0, 0};
      for (int l = g->D - 1; l >= 0; --l) {
        const int64_t j = rem % g->nv[l];
        rem /= g->nv[l];
        v[l] = oracle_cell_center(g->v_lo[l], g->v_hi[l], g->nv[l], j);
      }
      ksum_add(&s0, b[k]);
      for (int l = 0; l < g->D; ++l) ksum_add(&s1[l], b[k] * v[l]);
    }
    const double m0 = s0.s + s0.c;
    rho[ix] = dvol * m0;
    double u[3] = {0, 0, 0};
    for (int l = 0; l < g->D; ++l) u[l] = m0 != 0.0 ? (s1[l].s + s1[l].c) / m0 : 0.0;
    ksum_t s2[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t k = 0; k < nvs; ++k) {
      int64_t rem = k;
      for (int l = g->D - 1; l >= 0; --l) {
        const int64_t j = rem % g->nv[l];
        rem /= g->nv[l];
        const double d = oracle_cell_center(g->v_lo[l], g->v_hi[l], g->nv[l], j) - u[l];
        ksum_add(&s2[l], b[k] * d * d);
      }
    }
    for (int l = 0; l < g->D; ++l) {
      mean[l * nxs + ix] = u[l];
      disp[l * nxs + ix] = m0 != 0.0 ? (s2[l].s + s2[l].c) / m0 : 0.0;
    }
  }
}

/* Velocity distribution F(v) = dx^D sum_x f(x, v) (Sec. 3.3), prod(nv)
 * values; compensated, in x order. */
void oracle_velocity_distribution(const oracle_grid* g, const double* f, double* F) {
  int64_t nxs = 1, nvs = 1;
  double xvol = 1.0;
  for (int l = 0; l < g->D; ++l) {
    nxs *= g->nx[l];
    nvs *= g->nv[l];
    xvol *= (g->x_hi[l] - g->x_lo[l]) / (double)g->nx[l];
  }
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nvs; ++k) {
    ksum_t s = {0, 0};
    for (int64_t ix = 0; ix < nxs; ++ix) ksum_add(&s, f[ix * nvs + k]);
    F[k] = xvol * (s.s + s.c);
  }
}

/* rho(x) = Delta v^D * sum_v f, Eq. (poisson); compensated (Neumaier)
 * summation in index order. */
void oracle_density_moment(const oracle_grid* g, const double* f, double* rho) {
  const int64_t nxs = g->nx[0] * (g->D > 1 ? g->nx[1] : 1) * (g->D > 2 ? g->nx[2] : 1);
  int64_t nvs = 1;
  double dvol = 1.0;
  for (int l = 0; l < g->D; ++l) {
    nvs *= g->nv[l];
    dvol *= (g->v_hi[l] - g->v_lo[l]) / (double)g->nv[l];
  }
#pragma omp parallel for schedule(static)
  for (int64_t ix = 0; ix < nxs; ++ix) {
    const double* b = f + ix * nvs;
    double s = 0.0, comp = 0.0;
    for (int64_t k = 0; k < nvs; ++k) {
      double t = s + b[k];
      if (fabs(s) >= fabs(b[k]))
        comp += (s - t) + b[k];
      else
        comp += (b[k] - t) + s;
      s = t;
    }
    rho[ix] = dvol * (s + comp);
  }
}

/* exp(-2 pi i j k / n) with the angle reduced exactly: (j k) mod n */
static void twiddle(int64_t jk, int64_t n, int sign, double* c, double* s) {
  int64_t m = jk % n;
  double ang = 2.0 * M_PI * (double)m / (double)n;
  *c = cos(ang);
  *s = sign * sin(ang);
}

/* In-place complex DFT along axis `a` of a D-dim array (sizes dims),
 * q_k = sum_j q_j exp(sign * 2 pi i j k / n)  (App. C definition). */
static void dft_axis(double* re, double* im, const int64_t* dims, int D, int a,
                     int sign) {
  const int64_t outer = prod_range(dims, 0, a);
  const int64_t n = dims[a];
  const int64_t inner = prod_range(dims, a + 1, D);
#pragma omp parallel
  {
    double* tr = (double*)malloc(sizeof(double) * n);
    double* ti = (double*)malloc(sizeof(double) * n);
#pragma omp for schedule(static)
    for (int64_t p = 0; p < outer * inner; ++p) {
      int64_t o = p / inner, j0 = p % inner;
      double* br = re + o * n * inner + j0;
      double* bi = im + o * n * inner + j0;
      for (int64_t k = 0; k < n; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
          double c, s;
          twiddle(j * k, n, sign, &c, &s);
          double xr = br[j * inner], xi = bi[j * inner];
          sr += xr * c - xi * s;
          si += xr * s + xi * c;
        }
        tr[k] = sr;
        ti[k] = si;
      }
      for (int64_t k = 0; k < n; ++k) {
        br[k * inner] = tr[k];
        bi[k * inner] = ti[k];
      }
    }
    free(tr);
    free(ti);
  }
}

/* One-dimensional symbol of the discrete Laplacian times Delta^2, written
 * from the Green functions of Sec. 2.2 / App. C:
 *   order 2:  -4 sin^2(th/2)
 *   order 4:  [sin^2(th) - 16 sin^2(th/2)] / 3
 *   order 6: -[2 sin^2(3th/2) - 27 sin^2(th) + 270 sin^2(th/2)] / 45
 * so that G(k) = kappa / sum_l symbol(th_l)/Delta_l^2 reproduces
 * -pi G D^2/S2, 12 pi G D^2/S4 and -180 pi G D^2/S6 for kappa = 4 pi G. */
double oracle_laplacian_symbol(double th, int order) {
  double s1 = sin(th / 2.0), s2 = sin(th), s3 = sin(1.5 * th);
  if (order == 2) return -4.0 * s1 * s1;
  if (order == 4) return (s2 * s2 - 16.0 * s1 * s1) / 3.0;
  return -(2.0 * s3 * s3 - 27.0 * s2 * s2 + 270.0 * s1 * s1) / 45.0;
}

/* d(phi)/dx at cell i by the 2-, 4- or 6-point FDA of App. C (periodic),
 * the four-point form with the sign of the derivative (reading R7). */
static double fda(const double* phi, int64_t n, int64_t stride, int64_t i, double h,
                  int order) {
#define P(k) phi[((((i) + (k)) % n + n) % n) * stride]
  if (order == 2) return (P(1) - P(-1)) / (2.0 * h);
  if (order == 4) return (-P(2) + 8.0 * P(1) - 8.0 * P(-1) + P(-2)) / (12.0 * h);
  return (P(3) - 9.0 * P(2) + 45.0 * P(1) - 45.0 * P(-1) + 9.0 * P(-2) - P(-3)) /
         (60.0 * h);
#undef P
}

/* Periodic Poisson solve by the convolution method (Sec. 2.2), then
 * accel_l = -d phi / d x_l (FDA of the same order).  phi may be NULL.
 * accel holds D blocks of prod(nx) values. */
void oracle_poisson_solve(const oracle_grid* g, const double* rho, double* phi,
                          double* accel) {
  const int D = g->D;
  int64_t dims[3];
  int64_t nxs = 1;
  for (int l = 0; l < D; ++l) {
    dims[l] = g->nx[l];
    nxs *= g->nx[l];
  }
  double* re = (double*)malloc(sizeof(double) * nxs);
  double* im = (double*)malloc(sizeof(double) * nxs);
  double* ph = phi ? phi : (double*)malloc(sizeof(double) * nxs);
  for (int64_t i = 0; i < nxs; ++i) {
    re[i] = rho[i];
    im[i] = 0.0;
  }
  for (int a = 0; a < D; ++a) dft_axis(re, im, dims, D, a, -1);
  double h[3];
  for (int l = 0; l < D; ++l) h[l] = (g->x_hi[l] - g->x_lo[l]) / (double)g->nx[l];
  for (int64_t idx = 0; idx < nxs; ++idx) {
    int64_t rem = idx, kk[3] = {0, 0, 0};
    for (int l = D - 1; l >= 0; --l) {
      kk[l] = rem % dims[l];
      rem /= dims[l];
    }
    double L = 0.0;
    int zero = 1;
    for (int l = 0; l < D; ++l) {
      if (kk[l] != 0) zero = 0;
      double th = 2.0 * M_PI * (double)kk[l] / (double)dims[l]; /* k_l Delta_l */
      L += oracle_laplacian_symbol(th, g->poisson_order) / (h[l] * h[l]);
    }
    double G = zero ? 0.0 : g->kappa / L; /* reading R6 */
    re[idx] *= G;
    im[idx] *= G;
  }
  for (int a = 0; a < D; ++a) dft_axis(re, im, dims, D, a, +1);
  for (int64_t i = 0; i < nxs; ++i) ph[i] = re[i] / (double)nxs;
  for (int l = 0; l < D; ++l) {
    const int64_t inner = prod_range(dims, l + 1, D);
    const int64_t n = dims[l];
    for (int64_t idx = 0; idx < nxs; ++idx) {
      int64_t i = (idx / inner) % n;
      const double* base = ph + idx - i * inner;
      accel[l * nxs + idx] = -fda(base, n, inner, i, h[l], g->poisson_order);
    }
  }
  free(re);
  free(im);
  if (!phi) free(ph);
}

/* Integral of 1/r over the box [-a, a] x [-b, b] x [-c, c] (the potential
 * of a uniform box at its centre, per unit density): eight times the
 * octant integral, which has the closed form
 *   b c asinh(a / sqrt(b^2+c^2)) + a c asinh(b / sqrt(a^2+c^2))
 *   + a b asinh(c / sqrt(a^2+b^2)) - a^2/2 atan(b c / (a r))
 *   - b^2/2 atan(a c / (b r)) - c^2/2 atan(a b / (c r)),  r = |(a, b, c)|. */
double oracle_box_inverse_r(double a, double b, double c) {
  const double r = sqrt(a * a + b * b + c * c);
  const double oct = b * c * asinh(a / sqrt(b * b + c * c)) + a * c * asinh(b / sqrt(a * a + c * c)) +
                     a * b * asinh(c / sqrt(a * a + b * b)) - 0.5 * a * a * atan(b * c / (a * r)) -
                     0.5 * b * b * atan(a * c / (b * r)) - 0.5 * c * c * atan(a * b / (c * r));
  return 8.0 * oct;
}

/* Isolated-boundary field solve (reading R9), D = 3: phi = g * rho by the
 * DFT of the zero-padded density on the doubled grid, then the forces by
 * the FDA of order poisson_order on the doubled potential.  phi (may be
 * NULL) and accel as in oracle_poisson_solve. */
void oracle_poisson_isolated(const oracle_grid* g, const double* rho, double* phi,
                             double* accel) {
  int64_t n[3], m[3], nxs = 1, ms = 1;
  double h[3];
  for (int l = 0; l < 3; ++l) {
    n[l] = g->nx[l];
    m[l] = 2 * n[l];
    nxs *= n[l];
    ms *= m[l];
    h[l] = (g->x_hi[l] - g->x_lo[l]) / (double)g->nx[l];
  }
  double* re = (double*)calloc(ms, sizeof(double));
  double* im = (double*)calloc(ms, sizeof(double));
  double* gr = (double*)malloc(sizeof(double) * ms);
  double* gi = (double*)calloc(ms, sizeof(double));
  const double vol = h[0] * h[1] * h[2];
  /* padded density and the Green function times the cell volume */
  for (int64_t i = 0; i < n[0]; ++i)
    for (int64_t j = 0; j < n[1]; ++j)
      for (int64_t k = 0; k < n[2]; ++k)
        re[(i * m[1] + j) * m[2] + k] = rho[(i * n[1] + j) * n[2] + k];
  for (int64_t i = 0; i < m[0]; ++i)
    for (int64_t j = 0; j < m[1]; ++j)
      for (int64_t k = 0; k < m[2]; ++k) {
        const int64_t di = i < n[0] ? i : i - m[0];
        const int64_t dj = j < n[1] ? j : j - m[1];
        const int64_t dk = k < n[2] ? k : k - m[2];
        double inv_r;
        if (di == 0 && dj == 0 && dk == 0)
          inv_r = oracle_box_inverse_r(0.5 * h[0], 0.5 * h[1], 0.5 * h[2]) / vol;
        else
          inv_r = 1.0 / sqrt((di * h[0]) * (di * h[0]) + (dj * h[1]) * (dj * h[1]) +
                             (dk * h[2]) * (dk * h[2]));
        gr[(i * m[1] + j) * m[2] + k] = -g->kappa / (4.0 * M_PI) * inv_r * vol;
      }
  for (int a = 0; a < 3; ++a) {
    dft_axis(re, im, m, 3, a, -1);
    dft_axis(gr, gi, m, 3, a, -1);
  }
  for (int64_t q = 0; q < ms; ++q) {
    const double xr = re[q] * gr[q] - im[q] * gi[q];
    const double xi = re[q] * gi[q] + im[q] * gr[q];
    re[q] = xr;
    im[q] = xi;
  }
  for (int a = 0; a < 3; ++a) dft_axis(re, im, m, 3, a, +1);
  for (int64_t q = 0; q < ms; ++q) re[q] /= (double)ms; /* doubled potential */
  if (phi)
    for (int64_t i = 0; i < n[0]; ++i)
      for (int64_t j = 0; j < n[1]; ++j)
        for (int64_t k = 0; k < n[2]; ++k)
          phi[(i * n[1] + j) * n[2] + k] = re[(i * m[1] + j) * m[2] + k];
  for (int l = 0; l < 3; ++l) {
    const int64_t inner = prod_range(m, l + 1, 3);
    for (int64_t i = 0; i < n[0]; ++i)
      for (int64_t j = 0; j < n[1]; ++j)
        for (int64_t k = 0; k < n[2]; ++k) {
          const int64_t q = (i * m[1] + j) * m[2] + k;
          const int64_t pos = l == 0 ? i : (l == 1 ? j : k);
          accel[l * nxs + (i * n[1] + j) * n[2] + k] =
              -fda(re + q - pos * inner, m[l], inner, pos, h[l], g->poisson_order);
        }
  }
  free(re);
  free(im);
  free(gr);
  free(gi);
}

/* rho then Poisson: acceleration of the current f */
void oracle_field(const oracle_grid* g, const double* f, double* accel) {
  int64_t nxs = 1;
  for (int l = 0; l < g->D; ++l) nxs *= g->nx[l];
  double* rho = (double*)malloc(sizeof(double) * nxs);
  oracle_density_moment(g, f, rho);
  if (g->isolated)
    oracle_poisson_isolated(g, rho, NULL, accel);
  else
    oracle_poisson_solve(g, rho, NULL, accel);
  free(rho);
}

/* One time step by the directional splitting of Eq. (splitting):
 *   v1, v2, v3 (dt/2)  ->  x3, x2, x1 (dt)  ->  rho, Poisson  ->  v1, v2, v3 (dt/2)
 * accel: in = acceleration field belonging to f at entry, out = the field
 * computed after the physical-space block (Sec. 2.4). */
void oracle_step(const oracle_grid* g, double* f, double dt, double* accel) {
  int64_t nxs = 1;
  for (int l = 0; l < g->D; ++l) nxs *= g->nx[l];
  for (int l = 0; l < g->D; ++l) oracle_advect_v(g, f, l, 0.5 * dt, accel + l * nxs);
  for (int l = g->D - 1; l >= 0; --l) oracle_advect_x(g, f, l, dt);
  oracle_field(g, f, accel);
  for (int l = 0; l < g->D; ++l) oracle_advect_v(g, f, l, 0.5 * dt, accel + l * nxs);
}

/* nsteps Strang steps.  With merge_kicks the closing velocity half-step of
 * a step and the opening half-step of the next one, which use the same
 * acceleration, are taken as one velocity step with dt (the splitting of
 * Eq. (splitting) applied to consecutive steps); the first and the last
 * half-steps stay halves, so the result is at the same time level. */
void oracle_steps(const oracle_grid* g, double* f, double dt, int64_t nsteps, double* accel) {
  if (!g->merge_kicks) {
    for (int64_t k = 0; k < nsteps; ++k) oracle_step(g, f, dt, accel);
    return;
  }
  if (nsteps <= 0) return;
  int64_t nxs = 1;
  for (int l = 0; l < g->D; ++l) nxs *= g->nx[l];
  for (int l = 0; l < g->D; ++l) oracle_advect_v(g, f, l, 0.5 * dt, accel + l * nxs);
  for (int64_t k = 0; k < nsteps; ++k) {
    for (int l = g->D - 1; l >= 0; --l) oracle_advect_x(g, f, l, dt);
    oracle_field(g, f, accel);
    const double kick = k + 1 < nsteps ? dt : 0.5 * dt;
    for (int l = 0; l < g->D; ++l) oracle_advect_v(g, f, l, kick, accel + l * nxs);
  }
}

/* f = s(x) * g1(v1) * g2(v2) * g3(v3), the product taken left to right */
void oracle_init_separable(const oracle_grid* g, double* f, const double* s,
                           const double* g1, const double* g2, const double* g3) {
  int64_t nxs = 1, nvs = 1;
  for (int l = 0; l < g->D; ++l) {
    nxs *= g->nx[l];
    nvs *= g->nv[l];
  }
  const double* gv[3] = {g1, g2, g3};
#pragma omp parallel for schedule(static)
  for (int64_t ix = 0; ix < nxs; ++ix) {
    for (int64_t iv = 0; iv < nvs; ++iv) {
      int64_t rem = iv, jv[3] = {0, 0, 0};
      for (int l = g->D - 1; l >= 0; --l) {
        jv[l] = rem % g->nv[l];
        rem /= g->nv[l];
      }
      double val = s[ix];
      for (int l = 0; l < g->D; ++l) val = val * gv[l][jv[l]];
      f[ix * nvs + iv] = val;
    }
  }
}

/* Sum of f times the phase-space cell volume, index order, compensated */
double oracle_mass(const oracle_grid* g, const double* f) {
  int64_t ncell = 1;
  double vol = 1.0;
  for (int l = 0; l < g->D; ++l) {
    ncell *= g->nx[l] * g->nv[l];
    vol *= (g->x_hi[l] - g->x_lo[l]) / (double)g->nx[l];
    vol *= (g->v_hi[l] - g->v_lo[l]) / (double)g->nv[l];
  }
  double s = 0.0, comp = 0.0;
  for (int64_t k = 0; k < ncell; ++k) {
    double t = s + f[k];
    if (fabs(s) >= fabs(f[k]))
      comp += (s - t) + f[k];
    else
      comp += (f[k] - t) + s;
    s = t;
  }
  return vol * (s + comp);
}

int oracle_abi_version(void) { return 1; }

/* Threads of the OpenMP loops over pencils (for timing the oracle; the
 * pencils are independent, so the results do not depend on it). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
