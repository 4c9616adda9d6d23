/*
 * FP64 CPU oracle of the volume-based refined lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY: linked by nothing in the product path.  It shares
 * no code with the HIP library.
 *
 * Everything here is plain loops over index tables built (from the set
 * definitions of section 4) by tables.py:
 *
 *   equilibrium   eq. fequ  (incompressible, rho0 = 1)
 *   moments       eq. fvelocity, read as rho = sum f, u = sum e f / rho0
 *                 (the printed formula sums f^eq, which is circular; after a
 *                 collision both readings agree)
 *   collide       SRT:  f <- f - omega (f - f^eq)           (section 2)
 *                 or TRT with a constant body force (section 2, TRT
 *                 model and external forces): the even and odd parts of
 *                 f - f^eq relax with lambda_e and lambda_o, then
 *                 F_a = w_a rho0 (e_a . a) / c_s^2 is added; u in f^eq is
 *                 the unmodified sum e f / rho0
 *   explode       eq. ctof: every E_L cell takes its parent's 19 PDFs
 *   stream        pull: f(x) <- f(x - e_a) for x in I_L u H_L (eq. stream);
 *                 from a no-slip boundary cell: x's own opposite value
 *                 (halfway bounce-back, section 2.2)
 *   coalesce      eq. ftoc: 1/8 of the sum over the 8 children, for the
 *                 (cell, direction) pairs of the coalescence set
 *   step          Algorithm 1, NonUniformTimeStep(L), in the paper's order
 *
 * The equal-level Communication() of Algorithm 1 has no counterpart: cells are
 * addressed level-globally and periodicity is part of the index tables
 * (section 2.2: periodic boundaries are handled by the communication).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* D3Q19 (Qian, d'Humieres, Lallemand 1992): rest, 6 faces, 12 edges.
   Opposite directions adjacent.  Weights 1/3, 1/18, 1/36. */
static const int EV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double weight(int a) {
  if (a == 0) return 1.0 / 3.0;
  if (a <= 6) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

#define RHO0 1.0

typedef struct {
  int64_t n_int;    /* |I_L|: indices [0, n_int) are collided          */
  int64_t n_live;   /* |I_L u H_L|: indices [0, n_live) are streamed   */
  int64_t n_store;  /* |I_L u E_L|                                     */
  double *F;        /* n_store x 19, PDFs of the stored cells           */
  double *G;        /* n_live x 19, scratch for the pull                */
  const int32_t *pull;     /* n_live x 19: source index, -1 = fine region */
  const int32_t *expl_src; /* n_store - n_int: parent index in level L-1  */
  int64_t n_coal;
  const int32_t *coal_cell;   /* n_coal */
  const int32_t *coal_dir;    /* n_coal */
  const int32_t *coal_child;  /* n_coal x 8 */
  double omega;     /* SRT omega_L, or TRT lambda_e,L                  */
  int poison_far;   /* debug: overwrite E_L \ H_L with NaN after explosion */
  int trt;          /* 1: TRT + force collision with the two fields below */
  double lambda_o;  /* TRT odd rate lambda_o,L                          */
  double accel[3];  /* lattice acceleration a_L of this level           */
  int interp;       /* 1: interpolated explosion (the two tables below)  */
  const int32_t *expl_oct;  /* n_store - n_int x 3: octant of the cell in its parent */
  const int32_t *expl_nbr;  /* n_store - n_int x 6: parent's face neighbours in I_{L-1}, -1 none */
} orc_level;

void orc_lattice(int32_t *e, double *w) {
  for (int a = 0; a < Q; ++a) {
    for (int d = 0; d < 3; ++d) e[3 * a + d] = EV[a][d];
    w[a] = weight(a);
  }
}

/* eq. fequ with c = 1 in lattice units on every level */
static void feq_cell(double rho, const double u[3], double *out) {
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int a = 0; a < Q; ++a) {
    const double eu = EV[a][0] * u[0] + EV[a][1] * u[1] + EV[a][2] * u[2];
    out[a] = weight(a) * (rho + RHO0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
  }
}

static void moments_cell(const double *f, double *rho, double u[3]) {
  double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int a = 0; a < Q; ++a) {
    r += f[a];
    jx += EV[a][0] * f[a];
    jy += EV[a][1] * f[a];
    jz += EV[a][2] * f[a];
  }
  *rho = r;
  u[0] = jx / RHO0;
  u[1] = jy / RHO0;
  u[2] = jz / RHO0;
}

void orc_equilibrium(int64_t n, const double *rho, const double *u, double *feq) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) feq_cell(rho[i], u + 3 * i, feq + Q * i);
}

void orc_moments(int64_t n, const double *f, double *rho, double *u) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) moments_cell(f + Q * i, rho + i, u + 3 * i);
}

void orc_collide(int64_t n, double *f, double omega) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double rho, u[3], eq[Q];
    double *fi = f + Q * i;
    moments_cell(fi, &rho, u);
    feq_cell(rho, u, eq);
    for (int a = 0; a < Q; ++a) fi[a] = fi[a] - omega * (fi[a] - eq[a]);
  }
}

/* TRT collision with a body force, one cell after another: with abar the
   direction opposite to a, f+- = (f_a +- f_abar) / 2 and the same for f^eq,
   f_a <- f_a - lambda_e (f+ - f^eq+) - lambda_o (f- - f^eq-) + F_a,
   F_a = w_a rho0 (e_a . accel) / c_s^2 with c_s^2 = 1/3. */
void orc_collide_trt(int64_t n, double *f, double lambda_e, double lambda_o, const double accel[3]) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double rho, u[3], eq[Q], out[Q];
    double *fi = f + Q * i;
    moments_cell(fi, &rho, u);
    feq_cell(rho, u, eq);
    for (int a = 0; a < Q; ++a) {
      int ab = 0;  /* the opposite direction */
      while (EV[ab][0] != -EV[a][0] || EV[ab][1] != -EV[a][1] || EV[ab][2] != -EV[a][2]) ++ab;
      const double fp = 0.5 * (fi[a] + fi[ab]), fm = 0.5 * (fi[a] - fi[ab]);
      const double ep = 0.5 * (eq[a] + eq[ab]), em = 0.5 * (eq[a] - eq[ab]);
      const double ea = EV[a][0] * accel[0] + EV[a][1] * accel[1] + EV[a][2] * accel[2];
      out[a] = fi[a] - lambda_e * (fp - ep) - lambda_o * (fm - em) + weight(a) * RHO0 * ea * 3.0;
    }
    for (int a = 0; a < Q; ++a) fi[a] = out[a];
  }
}

static void collide(orc_level *lv) {
  if (lv->trt)
    orc_collide_trt(lv->n_int, lv->F, lv->omega, lv->lambda_o, lv->accel);
  else
    orc_collide(lv->n_int, lv->F, lv->omega);
}

/* minmod limiter: the smaller one-sided difference if both have the same
   sign, else 0 */
static double minmod(double p, double q) {
  if (p * q <= 0.0) return 0.0;
  return fabs(p) < fabs(q) ? p : q;
}

/* Explosion (section 4, eq. ctof): every cell of E_L takes its parent's 19
   values.  Interpolated form (the interpolation of exploded values of
   Algorithm 2, section 4.1; the scheme it cites is not given in the paper,
   so this is a reading): each PDF is reconstructed linearly inside the
   parent, f_a(x) = f_a(P) + sum_d (o_d - 1/2) / 2 g_d, o the octant of x in
   P, g_d the minmod-limited slope of f_a along axis d from P's two face
   neighbours (0 if either is not a level-(L-1) interior cell).  The 8
   children of a parent average to its values exactly, so mass and momentum
   are unchanged, and zero slopes give eq. ctof. */
static void explode(orc_level *lv, const orc_level *coarse) {
  const int64_t m = lv->n_store - lv->n_int;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    const double *src = coarse->F + Q * (int64_t)lv->expl_src[e];
    double *dst = lv->F + Q * (lv->n_int + e);
    for (int a = 0; a < Q; ++a) {
      double v = src[a];
      if (lv->interp) {
        for (int d = 0; d < 3; ++d) {
          const int32_t ip = lv->expl_nbr[6 * e + 2 * d], im = lv->expl_nbr[6 * e + 2 * d + 1];
          if (ip < 0 || im < 0) continue;
          const double g = minmod(coarse->F[Q * (int64_t)ip + a] - src[a], src[a] - coarse->F[Q * (int64_t)im + a]);
          v += (lv->expl_oct[3 * e + d] - 0.5) * 0.5 * g;
        }
      }
      dst[a] = v;
    }
  }
  if (lv->poison_far) {
    for (int64_t i = lv->n_live; i < lv->n_store; ++i)
      for (int a = 0; a < Q; ++a) lv->F[Q * i + a] = NAN;
  }
}

/* number of Stream(L) calls per level since the last reset (bookkeeping of
   the acoustic scaling: level L streams 2^L times per coarse step) */
#define ORC_MAX_LEVELS 16
static int64_t stream_calls[ORC_MAX_LEVELS];

void orc_stream_calls(int64_t *out, int num_levels, int reset) {
  for (int L = 0; L < num_levels && L < ORC_MAX_LEVELS; ++L) {
    out[L] = stream_calls[L];
    if (reset) stream_calls[L] = 0;
  }
}

/* the direction opposite to a */
static int opposite(int a) {
  int b = 0;
  while (EV[b][0] != -EV[a][0] || EV[b][1] != -EV[a][1] || EV[b][2] != -EV[a][2]) ++b;
  return b;
}

#define ORC_WALL (-2) /* pull source beyond a non-periodic end (tables.py) */

/* pull stream of I_L u H_L.  A source in a boundary cell (no-slip wall,
   section 2.2) holds, after the boundary treatment, the value x sent
   towards it reversed: x's own value of the opposite direction (halfway
   bounce-back). */
static void stream(orc_level *lv, int L) {
  if (L < ORC_MAX_LEVELS) stream_calls[L]++;
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lv->n_live; ++x) {
    for (int a = 0; a < Q; ++a) {
      const int32_t s = lv->pull[Q * x + a];
      lv->G[Q * x + a] = (s >= 0) ? lv->F[Q * (int64_t)s + a]
                         : (s == ORC_WALL ? lv->F[Q * x + opposite(a)] : NAN);
    }
  }
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lv->n_live; ++x)
    for (int a = 0; a < Q; ++a) lv->F[Q * x + a] = lv->G[Q * x + a];
}

static void coalesce(orc_level *lv, const orc_level *fine) {
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < lv->n_coal; ++p) {
    const int a = lv->coal_dir[p];
    double s = 0.0;
    for (int c = 0; c < 8; ++c) s += fine->F[Q * (int64_t)lv->coal_child[8 * p + c] + a];
    lv->F[Q * (int64_t)lv->coal_cell[p] + a] = s / 8.0;
  }
}

/* Algorithm 1, NonUniformTimeStep(L); level 0 is the coarsest level. */
static void step(orc_level *lv, int L, int Lmax) {
  collide(&lv[L]);
  if (L != Lmax) step(lv, L + 1, Lmax);
  if (L != 0) explode(&lv[L], &lv[L - 1]);
  stream(&lv[L], L);
  if (L != Lmax) coalesce(&lv[L], &lv[L + 1]);
  if (L == 0) return;
  collide(&lv[L]);
  if (L != Lmax) step(lv, L + 1, Lmax);
  stream(&lv[L], L);
  if (L != Lmax) coalesce(&lv[L], &lv[L + 1]);
}

void orc_coarse_steps(orc_level *levels, int num_levels, int steps) {
  for (int s = 0; s < steps; ++s) step(levels, 0, num_levels - 1);
}

/* the explosion of level L >= 1 alone, from the current level-(L-1) state
   (for tests of the exploded values) */
void orc_explode(orc_level *levels, int L) {
  if (L >= 1) explode(&levels[L], &levels[L - 1]);
}

int orc_sizeof_level(void) { return (int)sizeof(orc_level); }

/* threads of the OpenMP loops above (for timing the oracle on a given number
   of host cores); returns the previous maximum */
int orc_set_threads(int n) {
  const int prev = omp_get_max_threads();
  if (n > 0) omp_set_num_threads(n);
  return prev;
}
