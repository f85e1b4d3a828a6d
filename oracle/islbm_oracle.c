/*
 * ISLBM oracle -- plain, slow FP64 reference of one interpolation-supplemented
 * lattice Boltzmann time step for the side-heated cavity.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * loaded by the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark.  The product library never links, loads or calls it, and it
 * shares no source, header, table or helper with the HIP path.
 *
 * What it follows (Xu, Zhao, Xu & Jiang, "Interpolation-supplemented lattice
 * Boltzmann simulation of thermal convection on non-uniform meshes"):
 *   - Sec. 2.1, Eqs. (1)-(7): Boussinesq model; u_f, Ra, Pr fix nu, alpha, g*beta.
 *   - Sec. 2.1, Eq. (8) with the D2Q9/D3Q19 equilibrium moments, Guo's forcing
 *     moments M*F~, and rho/u definitions: MRT collision of f.
 *   - Sec. 2.1, Eq. (g) with the D2Q5/D3Q7 equilibrium moments and a_T: MRT
 *     collision of g.
 *   - Sec. 2.1, collision/streaming split (Eqs. collisionF ... streamingG).
 *   - Sec. 2.2, Fig. 1: streaming to the off-lattice points x + e_i dt, then
 *     quadratic interpolation back to the mesh nodes (He's scheme).
 *   - Sec. 2.3: half-way bounce-back (no-slip), half-way anti-bounce-back
 *     (isothermal walls, weights (4+a_T)/10 and (6+a_T)/21), half-way
 *     bounce-back for adiabatic walls.
 *   - Sec. 2.3, Eqs. (14), (erf), Table 1: meshes, lattice unit, H.
 *   - Sec. 2.3, Eqs. (16)-(18): wall derivative and midpoint-rule averages.
 *   - Sec. 3, Nu/Re definitions (volume, hot wall, centreline); Sec. 4 adds
 *     the cold wall.
 *
 * Readings taken where the paper is silent or garbled (each one is listed in
 * the design notes of the repository):
 *   - M, N, S, Q are not printed.  M and N are written here as the usual
 *     orthogonal polynomial bases (rows below); S uses s_e = s_eps (= s_pi)
 *     = s_nu and s_q (= s_m) = 8(2 - s_nu)/(8 - s_nu); Q uses q_j = 3 - sqrt(3)
 *     and q_e = q_nu = 4 sqrt(3) - 6.  Any rate can be overridden.
 *   - The last D2Q9 forcing moment is read as u F_y + v F_x (the printed
 *     u F_x + v F_y is inconsistent with Guo's force and with the D3Q19 form).
 *   - The interpolation stencil for node j is {j-1, j, j+1}, clamped to the
 *     fluid nodes, evaluated at the departure point x_j - e_i * Delta;
 *     a link that leaves the fluid region on any axis takes the wall rule.
 *   - Weights snap to one-hot when the departure point lies within
 *     1e-12 Delta of a stencil node.
 *   - Buoyancy reference T0 = (T_hot + T_cold)/2; force along +y.
 *
 * Precision: IEEE double throughout.  Plain loops; an optional OpenMP
 * "parallel for" over nodes is the only parallelism.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 19

typedef struct oracle {
  int dim, qf, qg;
  int n[3];               /* fluid nodes per axis (n[2] = 1 in 2-D) */
  double *x[3];           /* coordinates x_0 .. x_{N+1} per axis */
  double delta;           /* lattice unit: x_1 - x_0 */
  double heff[3];         /* wall-to-wall extent per axis */
  double H_lu;            /* characteristic length in lattice units (y) */
  double Ra, Pr, uf, Thot, Tcold, T0, dT;
  double nu, alpha, gbeta, aT, omega;
  int ef[QMAX][3], eg[7][3];
  int opp_f[QMAX], opp_g[7];
  double wf[QMAX];
  double M[QMAX][QMAX], Minv[QMAX][QMAX];
  double N[7][7], Ninv[7][7];
  double S[QMAX], Q[7];
  long nn;
  double *f, *g;          /* pre-collision populations f(x,t), [q][nn] */
  double *fp, *gp;        /* post-collision populations f+(x,t) */
  int collide_on;         /* 0: stream-only (collision is the identity) */
} oracle;

/* ------------------------------------------------------------------ */
/* Velocity sets (ordering is the interface ordering of populations).  */
/* ------------------------------------------------------------------ */
static const int E_D2Q9[9][3] = {
  {0,0,0},{1,0,0},{0,1,0},{-1,0,0},{0,-1,0},{1,1,0},{-1,1,0},{-1,-1,0},{1,-1,0}};
static const int E_D2Q5[5][3] = {{0,0,0},{1,0,0},{0,1,0},{-1,0,0},{0,-1,0}};
static const int E_D3Q19[19][3] = {
  {0,0,0},
  {1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1},
  {1,1,0},{-1,-1,0},{1,-1,0},{-1,1,0},
  {1,0,1},{-1,0,-1},{1,0,-1},{-1,0,1},
  {0,1,1},{0,-1,-1},{0,1,-1},{0,-1,1}};
static const int E_D3Q7[7][3] = {
  {0,0,0},{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1}};

/* Rows of the moment transform, written as polynomials of e (|e|^2 = s). */
static double row_d2q9(int r, int ex, int ey) {
  double s = ex * ex + ey * ey;
  switch (r) {
    case 0: return 1.0;                               /* rho     */
    case 1: return 3.0 * s - 4.0;                     /* e       */
    case 2: return 4.0 - 10.5 * s + 4.5 * s * s;      /* epsilon */
    case 3: return ex;                                /* j_x     */
    case 4: return (3.0 * s - 5.0) * ex;              /* q_x     */
    case 5: return ey;                                /* j_y     */
    case 6: return (3.0 * s - 5.0) * ey;              /* q_y     */
    case 7: return ex * ex - ey * ey;                 /* p_xx    */
    default: return ex * ey;                          /* p_xy    */
  }
}

static double row_d3q19(int r, int ex, int ey, int ez) {
  double s = ex * ex + ey * ey + ez * ez;
  double xx = ex * ex, yy = ey * ey, zz = ez * ez;
  switch (r) {
    case 0: return 1.0;
    case 1: return 19.0 * s - 30.0;
    case 2: return (21.0 * s * s - 53.0 * s + 24.0) / 2.0;
    case 3: return ex;
    case 4: return (5.0 * s - 9.0) * ex;
    case 5: return ey;
    case 6: return (5.0 * s - 9.0) * ey;
    case 7: return ez;
    case 8: return (5.0 * s - 9.0) * ez;
    case 9: return 3.0 * xx - s;
    case 10: return (3.0 * s - 5.0) * (3.0 * xx - s);
    case 11: return yy - zz;
    case 12: return (3.0 * s - 5.0) * (yy - zz);
    case 13: return ex * ey;
    case 14: return ey * ez;
    case 15: return ex * ez;
    case 16: return (yy - zz) * ex;
    case 17: return (zz - xx) * ey;
    default: return (xx - yy) * ez;
  }
}

static double row_d2q5(int r, int ex, int ey) {
  double s = ex * ex + ey * ey;
  switch (r) {
    case 0: return 1.0;
    case 1: return ex;
    case 2: return ey;
    case 3: return 5.0 * s - 4.0;
    default: return ex * ex - ey * ey;
  }
}

static double row_d3q7(int r, int ex, int ey, int ez) {
  double s = ex * ex + ey * ey + ez * ez;
  switch (r) {
    case 0: return 1.0;
    case 1: return ex;
    case 2: return ey;
    case 3: return ez;
    case 4: return 7.0 * s - 6.0;
    case 5: return 2.0 * ex * ex - ey * ey - ez * ez;
    default: return ey * ey - ez * ez;
  }
}

/* Gauss-Jordan inverse with partial pivoting; returns 0 on success. */
static int invert(int n, const double* a, double* inv) {
  double m[QMAX][2 * QMAX];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j)
      m[i][j] = (j < n) ? a[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(m[r][c]) > fabs(m[p][c])) p = r;
    if (fabs(m[p][c]) < 1e-300) return -1;
    if (p != c)
      for (int j = 0; j < 2 * n; ++j) { double t = m[p][j]; m[p][j] = m[c][j]; m[c][j] = t; }
    double d = m[c][c];
    for (int j = 0; j < 2 * n; ++j) m[c][j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double k = m[r][c];
      if (k == 0.0) continue;
      for (int j = 0; j < 2 * n; ++j) m[r][j] -= k * m[c][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) inv[i * n + j] = m[i][j + n];
  return 0;
}

/* Fills velocities, weights (f only) and the moment matrix of a lattice.
 * dim: 2 or 3; which: 0 = flow set (D2Q9/D3Q19), 1 = thermal set (D2Q5/D3Q7).
 * Returns q. */
int oracle_lattice(int dim, int which, int* e, double* w, double* mat) {
  int q;
  if (dim == 2 && which == 0) q = 9;
  else if (dim == 2) q = 5;
  else if (which == 0) q = 19;
  else q = 7;
  for (int i = 0; i < q; ++i) {
    const int* ei = (dim == 2) ? (which == 0 ? E_D2Q9[i] : E_D2Q5[i])
                               : (which == 0 ? E_D3Q19[i] : E_D3Q7[i]);
    if (e) for (int a = 0; a < 3; ++a) e[3 * i + a] = ei[a];
    if (w && which == 0) {
      int s = ei[0] * ei[0] + ei[1] * ei[1] + ei[2] * ei[2];
      if (dim == 2) w[i] = (s == 0) ? 4.0 / 9.0 : (s == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
      else w[i] = (s == 0) ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    if (mat)
      for (int r = 0; r < q; ++r) {
        double v;
        if (dim == 2) v = (which == 0) ? row_d2q9(r, ei[0], ei[1]) : row_d2q5(r, ei[0], ei[1]);
        else v = (which == 0) ? row_d3q19(r, ei[0], ei[1], ei[2]) : row_d3q7(r, ei[0], ei[1], ei[2]);
        mat[r * q + i] = v;
      }
  }
  return q;
}

/* ------------------------------------------------------------------ */
/* Meshes (Sec. 2.3): coordinates x_0..x_{N+1} in [.., ..], N fluid     */
/* nodes; the walls sit half-way between x_0,x_1 and x_N,x_{N+1}.       */
/*   kind 0: uniform, x_j = (j - 0.5)/N (Eq. 14, ghost mirrors at ends) */
/*   kind 1: error-function stretching (Eq. erf) with coefficient a     */
/*   kind 2: cosine,  x_j = (1 - cos(pi j/(N+1)))/2                     */
/*   kind 3: tanh,    x_j = (tanh(a(j/(N+1) - 1/2))/tanh(a/2) + 1)/2    */
/* ------------------------------------------------------------------ */
int oracle_mesh(int kind, int N, double a, double* x) {
  if (N < 3 || !x) return -1;
  for (int j = 0; j <= N + 1; ++j) {
    double xi = (double)j / (double)(N + 1);
    switch (kind) {
      case 0: x[j] = ((double)j - 0.5) / (double)N; break;
      case 1: x[j] = 0.5 * (erf(a * (xi - 0.5)) / erf(0.5 * a) + 1.0); break;
      case 2: x[j] = 0.5 * (1.0 - cos(M_PI * xi)); break;
      case 3: x[j] = 0.5 * (tanh(a * (xi - 0.5)) / tanh(0.5 * a) + 1.0); break;
      default: return -1;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Equilibrium and forcing moments (Sec. 2.1).                          */
/* ------------------------------------------------------------------ */
void oracle_meq(int dim, double rho, const double* u, double* m) {
  double ux = u[0], uy = u[1], uz = (dim == 3) ? u[2] : 0.0;
  double u2 = ux * ux + uy * uy + uz * uz;
  if (dim == 2) {
    double v[9] = {1.0, -2.0 + 3.0 * u2, 1.0 - 3.0 * u2, ux, -ux, uy, -uy,
                   ux * ux - uy * uy, ux * uy};
    for (int r = 0; r < 9; ++r) m[r] = rho * v[r];
  } else {
    double pxx = 2.0 * ux * ux - uy * uy - uz * uz, pww = uy * uy - uz * uz;
    double v[19] = {1.0, -11.0 + 19.0 * u2, 3.0 - 5.5 * u2,
                    ux, -2.0 / 3.0 * ux, uy, -2.0 / 3.0 * uy, uz, -2.0 / 3.0 * uz,
                    pxx, -0.5 * pxx, pww, -0.5 * pww,
                    ux * uy, uy * uz, ux * uz, 0.0, 0.0, 0.0};
    for (int r = 0; r < 19; ++r) m[r] = rho * v[r];
  }
}

/* Guo's forcing term in moment space, M F~ (Sec. 2.1). */
void oracle_mforce(int dim, const double* u, const double* F, double* m) {
  double ux = u[0], uy = u[1], uz = (dim == 3) ? u[2] : 0.0;
  double Fx = F[0], Fy = F[1], Fz = (dim == 3) ? F[2] : 0.0;
  double uF = ux * Fx + uy * Fy + uz * Fz;
  if (dim == 2) {
    double v[9] = {0.0, 6.0 * uF, -6.0 * uF, Fx, -Fx, Fy, -Fy,
                   2.0 * ux * Fx - 2.0 * uy * Fy, ux * Fy + uy * Fx};
    for (int r = 0; r < 9; ++r) m[r] = v[r];
  } else {
    double v[19] = {0.0, 38.0 * uF, -11.0 * uF,
                    Fx, -2.0 / 3.0 * Fx, Fy, -2.0 / 3.0 * Fy, Fz, -2.0 / 3.0 * Fz,
                    4.0 * ux * Fx - 2.0 * uy * Fy - 2.0 * uz * Fz,
                    -2.0 * ux * Fx + uy * Fy + uz * Fz,
                    2.0 * uy * Fy - 2.0 * uz * Fz,
                    -uy * Fy + uz * Fz,
                    ux * Fy + uy * Fx, uy * Fz + uz * Fy, ux * Fz + uz * Fx,
                    0.0, 0.0, 0.0};
    for (int r = 0; r < 19; ++r) m[r] = v[r];
  }
}

/* Thermal equilibrium moments n^eq (Sec. 2.1). */
void oracle_neq(int dim, double aT, double T, const double* u, double* n) {
  if (dim == 2) {
    double v[5] = {T, u[0] * T, u[1] * T, aT * T, 0.0};
    for (int r = 0; r < 5; ++r) n[r] = v[r];
  } else {
    double v[7] = {T, u[0] * T, u[1] * T, u[2] * T, aT * T, 0.0, 0.0};
    for (int r = 0; r < 7; ++r) n[r] = v[r];
  }
}

/* ------------------------------------------------------------------ */
/* Context                                                              */
/* ------------------------------------------------------------------ */
static int opposite(const int (*e)[3], int q, int i) {
  for (int k = 0; k < q; ++k)
    if (e[k][0] == -e[i][0] && e[k][1] == -e[i][1] && e[k][2] == -e[i][2]) return k;
  return -1;
}

void oracle_destroy(oracle* o);

oracle* oracle_create(int dim, const int* n, const double* x0, const double* x1,
                      const double* x2, double Ra, double Pr, double uf,
                      double Thot, double Tcold) {
  if (dim != 2 && dim != 3) return NULL;
  oracle* o = (oracle*)calloc(1, sizeof(oracle));
  o->dim = dim;
  o->qf = (dim == 2) ? 9 : 19;
  o->qg = (dim == 2) ? 5 : 7;
  const double* xs[3] = {x0, x1, x2};
  o->nn = 1;
  for (int a = 0; a < 3; ++a) {
    o->n[a] = (a < dim) ? n[a] : 1;
    if (a < dim) {
      o->x[a] = (double*)malloc(sizeof(double) * (o->n[a] + 2));
      memcpy(o->x[a], xs[a], sizeof(double) * (o->n[a] + 2));
      o->heff[a] = 0.5 * (o->x[a][o->n[a]] + o->x[a][o->n[a] + 1]) - 0.5 * (o->x[a][0] + o->x[a][1]);
    } else {
      o->heff[a] = 1.0;
    }
    o->nn *= o->n[a];
  }
  o->delta = o->x[0][1] - o->x[0][0];
  /* One lattice unit on every axis (shared time step); ghost spacings at
   * both ends equal it and no interior spacing is smaller. */
  for (int a = 0; a < dim; ++a) {
    int na = o->n[a];
    /* differences of coordinates carry the rounding of their magnitude */
    double tol = 1e-12 * o->delta +
                 16.0 * 2.220446049250313e-16 * (fabs(o->x[a][0]) + fabs(o->x[a][na + 1]));
    double d0 = o->x[a][1] - o->x[a][0], d1 = o->x[a][na + 1] - o->x[a][na];
    int bad = fabs(d0 - o->delta) > tol || fabs(d1 - o->delta) > tol;
    for (int j = 0; j <= na; ++j)
      if (o->x[a][j + 1] - o->x[a][j] < o->delta - tol) bad = 1;
    if (bad || na < 3) { oracle_destroy(o); return NULL; }
  }
  o->H_lu = o->heff[1] / o->delta;     /* Table 1: characteristic length */
  o->Ra = Ra; o->Pr = Pr;
  o->uf = (uf > 0.0) ? uf : 0.1 / sqrt(3.0);   /* Ma = u_f / c_s = 0.1 */
  o->Thot = Thot; o->Tcold = Tcold;
  o->T0 = 0.5 * (Thot + Tcold);
  o->dT = Thot - Tcold;
  double dTs = (o->dT != 0.0) ? o->dT : 1.0;
  /* u_f = sqrt(g beta H dT) (Eq. 2 scalings); Eqs. (5)-(6) coefficients. */
  o->gbeta = o->uf * o->uf / (o->H_lu * dTs);
  o->nu = o->uf * o->H_lu * sqrt(Pr / Ra);
  o->alpha = o->uf * o->H_lu / sqrt(Ra * Pr);
  o->aT = (dim == 2) ? 20.0 * sqrt(3.0) * o->alpha - 4.0 : 42.0 * sqrt(3.0) * o->alpha - 6.0;
  o->omega = (dim == 2) ? (4.0 + o->aT) / 10.0 : (6.0 + o->aT) / 21.0;

  int ef[QMAX * 3], eg[7 * 3];
  double Mf[QMAX * QMAX], Ng[49];
  oracle_lattice(dim, 0, ef, o->wf, Mf);
  oracle_lattice(dim, 1, eg, NULL, Ng);
  for (int i = 0; i < o->qf; ++i) for (int a = 0; a < 3; ++a) o->ef[i][a] = ef[3 * i + a];
  for (int i = 0; i < o->qg; ++i) for (int a = 0; a < 3; ++a) o->eg[i][a] = eg[3 * i + a];
  for (int i = 0; i < o->qf; ++i) o->opp_f[i] = opposite((const int (*)[3])o->ef, o->qf, i);
  for (int i = 0; i < o->qg; ++i) o->opp_g[i] = opposite((const int (*)[3])o->eg, o->qg, i);
  double Mi[QMAX * QMAX], Ni[49];
  invert(o->qf, Mf, Mi);
  invert(o->qg, Ng, Ni);
  for (int r = 0; r < o->qf; ++r)
    for (int c = 0; c < o->qf; ++c) { o->M[r][c] = Mf[r * o->qf + c]; o->Minv[r][c] = Mi[r * o->qf + c]; }
  for (int r = 0; r < o->qg; ++r)
    for (int c = 0; c < o->qg; ++c) { o->N[r][c] = Ng[r * o->qg + c]; o->Ninv[r][c] = Ni[r * o->qg + c]; }

  /* Relaxation rates (reading; see header). */
  double snu = 1.0 / (3.0 * o->nu + 0.5);
  double sq = 8.0 * (2.0 - snu) / (8.0 - snu);
  if (dim == 2) {
    double s[9] = {1.0, snu, snu, 1.0, sq, 1.0, sq, snu, snu};
    for (int r = 0; r < 9; ++r) o->S[r] = s[r];
  } else {
    double s[19] = {1.0, snu, snu, 1.0, sq, 1.0, sq, 1.0, sq,
                    snu, snu, snu, snu, snu, snu, snu, sq, sq, sq};
    for (int r = 0; r < 19; ++r) o->S[r] = s[r];
  }
  double qj = 3.0 - sqrt(3.0), qe = 4.0 * sqrt(3.0) - 6.0;
  if (dim == 2) {
    double q[5] = {1.0, qj, qj, qe, qe};
    for (int r = 0; r < 5; ++r) o->Q[r] = q[r];
  } else {
    double q[7] = {1.0, qj, qj, qj, qe, qe, qe};
    for (int r = 0; r < 7; ++r) o->Q[r] = q[r];
  }
  o->collide_on = 1;

  o->f = (double*)calloc((size_t)o->qf * o->nn, sizeof(double));
  o->fp = (double*)calloc((size_t)o->qf * o->nn, sizeof(double));
  o->g = (double*)calloc((size_t)o->qg * o->nn, sizeof(double));
  o->gp = (double*)calloc((size_t)o->qg * o->nn, sizeof(double));
  /* Start at rest with T = 0 inside: f_i = w_i (rho = 1), g_i = 0. */
  for (int i = 0; i < o->qf; ++i)
    for (long k = 0; k < o->nn; ++k) o->f[(size_t)i * o->nn + k] = o->wf[i];
  return o;
}

void oracle_destroy(oracle* o) {
  if (!o) return;
  for (int a = 0; a < 3; ++a) free(o->x[a]);
  free(o->f); free(o->g); free(o->fp); free(o->gp);
  free(o);
}

/* out: delta, H_lu, nu, alpha, gbeta, aT, omega, uf, T0, s_nu */
void oracle_params(const oracle* o, double* out) {
  out[0] = o->delta; out[1] = o->H_lu; out[2] = o->nu; out[3] = o->alpha;
  out[4] = o->gbeta; out[5] = o->aT; out[6] = o->omega; out[7] = o->uf;
  out[8] = o->T0; out[9] = (o->dim == 2) ? o->S[7] : o->S[9];   /* s_nu (stress row) */
}

/* Overrides: rates S (qf entries), Q (qg entries), g*beta; NULL keeps. */
void oracle_override(oracle* o, const double* S, const double* Q, const double* gbeta,
                     int collide_on) {
  if (S) for (int r = 0; r < o->qf; ++r) o->S[r] = S[r];
  if (Q) for (int r = 0; r < o->qg; ++r) o->Q[r] = Q[r];
  if (gbeta) o->gbeta = *gbeta;
  o->collide_on = collide_on;
}

void oracle_get_rates(const oracle* o, double* S, double* Q) {
  for (int r = 0; r < o->qf; ++r) S[r] = o->S[r];
  for (int r = 0; r < o->qg; ++r) Q[r] = o->Q[r];
}

void oracle_set_state(oracle* o, const double* f, const double* g) {
  memcpy(o->f, f, sizeof(double) * o->qf * o->nn);
  memcpy(o->g, g, sizeof(double) * o->qg * o->nn);
}
void oracle_get_state(const oracle* o, double* f, double* g) {
  if (f) memcpy(f, o->f, sizeof(double) * o->qf * o->nn);
  if (g) memcpy(g, o->g, sizeof(double) * o->qg * o->nn);
}
void oracle_set_post(oracle* o, const double* fp, const double* gp) {
  memcpy(o->fp, fp, sizeof(double) * o->qf * o->nn);
  memcpy(o->gp, gp, sizeof(double) * o->qg * o->nn);
}
void oracle_get_post(const oracle* o, double* fp, double* gp) {
  if (fp) memcpy(fp, o->fp, sizeof(double) * o->qf * o->nn);
  if (gp) memcpy(gp, o->gp, sizeof(double) * o->qg * o->nn);
}

/* ------------------------------------------------------------------ */
/* Macroscopic quantities of one node (Sec. 2.1): rho = sum f,          */
/* T = sum g, F = rho g beta (T - T0) y^, u = (sum e f + F/2)/rho.      */
/* ------------------------------------------------------------------ */
static void macro(const oracle* o, const double* f, const double* g, double* rho,
                  double* u, double* T, double* F) {
  double r = 0.0, j[3] = {0.0, 0.0, 0.0}, t = 0.0;
  for (int i = 0; i < o->qf; ++i) {
    r += f[i];
    for (int a = 0; a < 3; ++a) j[a] += o->ef[i][a] * f[i];
  }
  for (int i = 0; i < o->qg; ++i) t += g[i];
  F[0] = 0.0; F[1] = r * o->gbeta * (t - o->T0); F[2] = 0.0;
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / r;
  *rho = r; *T = t;
}

/* Collision of one node: m+ = m - S(m - m^eq) + (I - S/2) M F~, f+ = M^-1 m+;
 * n+ = n - Q(n - n^eq), g+ = N^-1 n+. */
void oracle_collide_node(const oracle* o, const double* f, const double* g,
                         double* fo, double* go) {
  if (!o->collide_on) {
    for (int i = 0; i < o->qf; ++i) fo[i] = f[i];
    for (int i = 0; i < o->qg; ++i) go[i] = g[i];
    return;
  }
  double rho, u[3], T, F[3];
  macro(o, f, g, &rho, u, &T, F);
  double m[QMAX], meq[QMAX], mF[QMAX], mp[QMAX];
  for (int r = 0; r < o->qf; ++r) {
    m[r] = 0.0;
    for (int i = 0; i < o->qf; ++i) m[r] += o->M[r][i] * f[i];
  }
  oracle_meq(o->dim, rho, u, meq);
  oracle_mforce(o->dim, u, F, mF);
  for (int r = 0; r < o->qf; ++r)
    mp[r] = m[r] - o->S[r] * (m[r] - meq[r]) + (1.0 - 0.5 * o->S[r]) * mF[r];
  for (int i = 0; i < o->qf; ++i) {
    fo[i] = 0.0;
    for (int r = 0; r < o->qf; ++r) fo[i] += o->Minv[i][r] * mp[r];
  }
  double n[7], neq[7], np[7];
  for (int r = 0; r < o->qg; ++r) {
    n[r] = 0.0;
    for (int i = 0; i < o->qg; ++i) n[r] += o->N[r][i] * g[i];
  }
  oracle_neq(o->dim, o->aT, T, u, neq);
  for (int r = 0; r < o->qg; ++r) np[r] = n[r] - o->Q[r] * (n[r] - neq[r]);
  for (int i = 0; i < o->qg; ++i) {
    go[i] = 0.0;
    for (int r = 0; r < o->qg; ++r) go[i] += o->Ninv[i][r] * np[r];
  }
}

void oracle_collide(oracle* o) {
  long nn = o->nn;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < nn; ++k) {
    double f[QMAX], g[7], fo[QMAX], go[7];
    for (int i = 0; i < o->qf; ++i) f[i] = o->f[(size_t)i * nn + k];
    for (int i = 0; i < o->qg; ++i) g[i] = o->g[(size_t)i * nn + k];
    oracle_collide_node(o, f, g, fo, go);
    for (int i = 0; i < o->qf; ++i) o->fp[(size_t)i * nn + k] = fo[i];
    for (int i = 0; i < o->qg; ++i) o->gp[(size_t)i * nn + k] = go[i];
  }
}

/* ------------------------------------------------------------------ */
/* Quadratic (3-point Lagrange) interpolation (Sec. 2.2).               */
/* ------------------------------------------------------------------ */
void oracle_lagrange3(const double* xs, double xd, double delta, double* w) {
  for (int k = 0; k < 3; ++k)
    if (fabs(xd - xs[k]) <= 1e-12 * delta) {
      w[0] = w[1] = w[2] = 0.0;
      w[k] = 1.0;
      return;
    }
  w[0] = (xd - xs[1]) * (xd - xs[2]) / ((xs[0] - xs[1]) * (xs[0] - xs[2]));
  w[1] = (xd - xs[0]) * (xd - xs[2]) / ((xs[1] - xs[0]) * (xs[1] - xs[2]));
  w[2] = (xd - xs[0]) * (xd - xs[1]) / ((xs[2] - xs[0]) * (xs[2] - xs[1]));
}

/* Stencil of fluid node idx (0-based) on axis a for lattice direction s:
 * base b (0-based first node of {b, b+1, b+2}) and the three weights at the
 * departure point x_idx - s*Delta. */
static void stencil(const oracle* o, int a, int idx, int s, int* b, double* w) {
  int n = o->n[a];
  int lo = idx - 1;
  if (lo < 0) lo = 0;
  if (lo > n - 3) lo = n - 3;
  const double* x = o->x[a] + 1;   /* x[k] = coordinate of fluid node k */
  double xd = x[idx] - (double)s * o->delta;
  *b = lo;
  oracle_lagrange3(x + lo, xd, o->delta, w);
}

/* Pull one node of population p of a set (f or g) from post-collision
 * arrays src ([q][nn]); returns f_p(x, t+1). */
static double pull(const oracle* o, int isg, const double* src, int p, const int* idx) {
  const int (*e)[3] = isg ? (const int (*)[3])o->eg : (const int (*)[3])o->ef;
  const int* opp = isg ? o->opp_g : o->opp_f;
  long nn = o->nn;
  long node = idx[0] + (long)o->n[0] * (idx[1] + (long)o->n[1] * idx[2]);
  /* Wall rules: the link leaves the fluid on some axis. */
  int cross = 0, xwall = 0;
  double Tw = 0.0;
  for (int a = 0; a < o->dim; ++a) {
    if (e[p][a] == 1 && idx[a] == 0) {
      cross = 1;
      if (a == 0) { xwall = 1; Tw = o->Thot; }
    }
    if (e[p][a] == -1 && idx[a] == o->n[a] - 1) {
      cross = 1;
      if (a == 0) { xwall = 1; Tw = o->Tcold; }
    }
  }
  if (cross) {
    double back = src[(size_t)opp[p] * nn + node];
    if (isg && xwall) return -back + o->omega * Tw;  /* anti-bounce-back */
    return back;                                      /* bounce-back */
  }
  /* Tensor product of 1-D quadratic interpolation over the shifted axes. */
  int b[3];
  double w[3][3];
  int len[3];
  for (int a = 0; a < 3; ++a) {
    if (a < o->dim && e[p][a] != 0) {
      stencil(o, a, idx[a], e[p][a], &b[a], w[a]);
      len[a] = 3;
    } else {
      b[a] = idx[a];
      w[a][0] = 1.0;
      len[a] = 1;
    }
  }
  double sum = 0.0;
  for (int c = 0; c < len[2]; ++c)
    for (int bb = 0; bb < len[1]; ++bb)
      for (int aa = 0; aa < len[0]; ++aa) {
        long k = (b[0] + aa) + (long)o->n[0] * ((b[1] + bb) + (long)o->n[1] * (b[2] + c));
        sum += w[0][aa] * w[1][bb] * w[2][c] * src[(size_t)p * nn + k];
      }
  return sum;
}

/* Stream one node from external post-collision arrays fp, gp. */
void oracle_stream_node(const oracle* o, const double* fp, const double* gp, long node,
                        double* fo, double* go) {
  int idx[3];
  idx[0] = (int)(node % o->n[0]);
  idx[1] = (int)((node / o->n[0]) % o->n[1]);
  idx[2] = (int)(node / ((long)o->n[0] * o->n[1]));
  for (int p = 0; p < o->qf; ++p) fo[p] = pull(o, 0, fp, p, idx);
  for (int p = 0; p < o->qg; ++p) go[p] = pull(o, 1, gp, p, idx);
}

void oracle_stream(oracle* o) {
  long nn = o->nn;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < nn; ++k) {
    double fo[QMAX], go[7];
    oracle_stream_node(o, o->fp, o->gp, k, fo, go);
    for (int i = 0; i < o->qf; ++i) o->f[(size_t)i * nn + k] = fo[i];
    for (int i = 0; i < o->qg; ++i) o->g[(size_t)i * nn + k] = go[i];
  }
}

/* nsteps x (collide, stream): f(t) -> f(t + nsteps). */
void oracle_run(oracle* o, long nsteps) {
  for (long s = 0; s < nsteps; ++s) {
    oracle_collide(o);
    oracle_stream(o);
  }
}

/* One step at selected nodes from external post-collision state:
 * stream to t+1, then collide; out arrays are [count][q]. */
void oracle_sample_step(const oracle* o, const double* fp, const double* gp,
                        const long* nodes, long count, double* fout, double* gout) {
#pragma omp parallel for schedule(static)
  for (long s = 0; s < count; ++s) {
    double f[QMAX], g[7];
    oracle_stream_node(o, fp, gp, nodes[s], f, g);
    oracle_collide_node(o, f, g, fout + (size_t)s * o->qf, gout + (size_t)s * o->qg);
  }
}

/* Macroscopic fields of the pre-collision state: rho, u (incl. F/2), T. */
void oracle_fields(const oracle* o, double* rho, double* ux, double* uy, double* uz, double* T) {
  long nn = o->nn;
  for (long k = 0; k < nn; ++k) {
    double f[QMAX], g[7], r, u[3], t, F[3];
    for (int i = 0; i < o->qf; ++i) f[i] = o->f[(size_t)i * nn + k];
    for (int i = 0; i < o->qg; ++i) g[i] = o->g[(size_t)i * nn + k];
    macro(o, f, g, &r, u, &t, F);
    if (rho) rho[k] = r;
    if (ux) ux[k] = u[0];
    if (uy) uy[k] = u[1];
    if (uz) uz[k] = u[2];
    if (T) T[k] = t;
  }
}

/* ------------------------------------------------------------------ */
/* Diagnostics (Sec. 2.3 Eqs. 16-18, Sec. 3 and 4 definitions).         */
/* ------------------------------------------------------------------ */

/* One-sided wall derivative, Eq. (17) (reduces to Eq. (16) at q = 1),
 * in lattice units.  top = 0: bottom/low wall (phi1 = node 1, phi2 = node 2);
 * top = 1: top/high wall (phi1 = node N, phi2 = node N-1). */
double oracle_wall_derivative(int top, double q, double phiw, double phi1, double phi2) {
  double num = -4.0 * q * (q + 1.0) * phiw + (2.0 * q + 1.0) * (2.0 * q + 1.0) * phi1 - phi2;
  double d = num / (q * (2.0 * q + 1.0));
  return top ? -d : d;
}

/* Midpoint-rule weight of node k (0-based) on axis a, Eq. (18):
 * (x_{k+1} - x_{k-1})/2 with the ghost coordinates at the ends. */
static double vol(const oracle* o, int a, int k) {
  if (a >= o->dim) return 1.0;
  const double* x = o->x[a];
  return 0.5 * (x[k + 2] - x[k]);
}

/* Weights of the value and x-derivative at the mid-plane x = x_c from the
 * quadratic through the three nodes nearest x_c (average of the two
 * quadratics when two choices tie).  Writes up to 4 (node, cv, cd). */
static int midline(const oracle* o, int* nodes, double* cv, double* cd) {
  int n = o->n[0];
  const double* x = o->x[0] + 1;
  double xc = 0.5 * (0.5 * (o->x[0][0] + o->x[0][1]) + 0.5 * (o->x[0][n] + o->x[0][n + 1]));
  int k = 0;
  for (int i = 1; i < n; ++i)
    if (fabs(x[i] - xc) < fabs(x[k] - xc) - 1e-12 * o->delta) k = i;
  /* candidate triples */
  int starts[2], ns = 0;
  int lo = k - 1;
  if (lo < 0) lo = 0;
  if (lo > n - 3) lo = n - 3;
  /* tie: xc exactly between node k and k+1 */
  if (k + 1 < n && fabs(fabs(x[k + 1] - xc) - fabs(x[k] - xc)) <= 1e-12 * o->delta) {
    int l0 = k - 1, l1 = k;
    if (l0 < 0) l0 = 0;
    if (l1 > n - 3) l1 = n - 3;
    starts[ns++] = l0;
    if (l1 != l0) starts[ns++] = l1;
  } else {
    starts[ns++] = lo;
  }
  int cnt = 0;
  for (int i = 0; i < 4; ++i) { nodes[i] = 0; cv[i] = 0.0; cd[i] = 0.0; }
  int base = starts[0];
  for (int s = 0; s < ns; ++s) {
    const double* xs = x + starts[s];
    double w[3], d[3];
    oracle_lagrange3(xs, xc, o->delta, w);
    /* derivative of the Lagrange basis at xc */
    d[0] = ((xc - xs[1]) + (xc - xs[2])) / ((xs[0] - xs[1]) * (xs[0] - xs[2]));
    d[1] = ((xc - xs[0]) + (xc - xs[2])) / ((xs[1] - xs[0]) * (xs[1] - xs[2]));
    d[2] = ((xc - xs[0]) + (xc - xs[1])) / ((xs[2] - xs[0]) * (xs[2] - xs[1]));
    for (int j = 0; j < 3; ++j) {
      int slot = starts[s] + j - base;
      cv[slot] += w[j] / ns;
      cd[slot] += d[j] / ns;
    }
  }
  cnt = starts[ns - 1] + 3 - base;
  for (int i = 0; i < cnt; ++i) nodes[i] = base + i;
  return cnt;
}

/* Statistics of the pre-collision state f(t), g(t).  out[]:
 *  0 <Nu>_V, 1 Nu_hot, 2 Nu_cold, 3 Nu_middle, 4 <Re>_V (|u| over all
 *  components), 5 <Re>_V with sqrt(u^2+v^2) only, 6 mass sum rho*V/Delta^d,
 *  7 sum rho, 8 max|u*|, 9 max|v*|, 10 max|w*|, 11 non-finite count,
 *  12 <Re> of the root-mean-square velocity, sqrt(Ra/Pr) sqrt(<|u*|^2>_V). */
void oracle_stats(const oracle* o, double* out) {
  long nn = o->nn;
  int dim = o->dim;
  double* rho = (double*)malloc(sizeof(double) * nn);
  double* ux = (double*)malloc(sizeof(double) * nn);
  double* uy = (double*)malloc(sizeof(double) * nn);
  double* uz = (double*)malloc(sizeof(double) * nn);
  double* T = (double*)malloc(sizeof(double) * nn);
  oracle_fields(o, rho, ux, uy, uz, T);
  double dTs = (o->dT != 0.0) ? o->dT : 1.0;
  double sRaPr = sqrt(o->Ra * o->Pr), sRaoPr = sqrt(o->Ra / o->Pr);
  double nuv = 0.0, re = 0.0, re2 = 0.0, mass = 0.0, msum = 0.0, rms = 0.0;
  double umax = 0.0, vmax = 0.0, wmax = 0.0, bad = 0.0;
  int n0 = o->n[0], n1 = o->n[1], n2 = o->n[2];
  double dd = (dim == 2) ? o->delta * o->delta : o->delta * o->delta * o->delta;
  for (int k = 0; k < n2; ++k)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n0; ++i) {
        long c = i + (long)n0 * (j + (long)n1 * k);
        double V = vol(o, 0, i) * vol(o, 1, j) * vol(o, 2, k);
        double W = V / (o->heff[0] * o->heff[1] * o->heff[2]);
        double us = ux[c] / o->uf, vs = uy[c] / o->uf, ws = uz[c] / o->uf;
        double Ts = (T[c] - o->T0) / dTs;
        nuv += W * us * Ts;
        re += W * sqrt(us * us + vs * vs + ws * ws);
        re2 += W * sqrt(us * us + vs * vs);
        rms += W * (us * us + vs * vs + ws * ws);
        mass += rho[c] * V / dd;
        msum += rho[c];
        if (fabs(us) > umax) umax = fabs(us);
        if (fabs(vs) > vmax) vmax = fabs(vs);
        if (fabs(ws) > wmax) wmax = fabs(ws);
        if (!isfinite(rho[c]) || !isfinite(ux[c]) || !isfinite(uy[c]) || !isfinite(uz[c]) ||
            !isfinite(T[c]))
          bad += 1.0;
      }
  /* Wall Nusselt numbers: line (2-D) or area (3-D) averages of -dT_star/dx_star. */
  double qh = (o->x[0][2] - o->x[0][1]) / o->delta;
  double qc = (o->x[0][n0] - o->x[0][n0 - 1]) / o->delta;
  double Thot_s = (o->Thot - o->T0) / dTs, Tcold_s = (o->Tcold - o->T0) / dTs;
  double nuh = 0.0, nuc = 0.0, num = 0.0;
  int mn[4];
  double mcv[4], mcd[4];
  int mc = midline(o, mn, mcv, mcd);
  for (int k = 0; k < n2; ++k)
    for (int j = 0; j < n1; ++j) {
      double A = vol(o, 1, j) * vol(o, 2, k) / (o->heff[1] * o->heff[2]);
      long r0 = (long)n0 * (j + (long)n1 * k);
      double T1 = (T[r0 + 0] - o->T0) / dTs, T2 = (T[r0 + 1] - o->T0) / dTs;
      double TN = (T[r0 + n0 - 1] - o->T0) / dTs, TN1 = (T[r0 + n0 - 2] - o->T0) / dTs;
      double dh = oracle_wall_derivative(0, qh, Thot_s, T1, T2) * o->H_lu;
      double dc = oracle_wall_derivative(1, qc, Tcold_s, TN, TN1) * o->H_lu;
      nuh += -A * dh;
      nuc += -A * dc;
      double conv = 0.0, der = 0.0;
      for (int m = 0; m < mc; ++m) {
        long c = r0 + mn[m];
        double Ts = (T[c] - o->T0) / dTs;
        conv += mcv[m] * (ux[c] / o->uf) * Ts;
        der += mcd[m] * Ts;
      }
      /* der is d/dx in coordinate units; dx* = dx / heff_y (the height H) */
      num += A * (sRaPr * conv - der * o->heff[1]);
    }
  out[0] = sRaPr * nuv + 1.0;
  out[1] = nuh;
  out[2] = nuc;
  out[3] = num;
  out[4] = sRaoPr * re;
  out[5] = sRaoPr * re2;
  out[6] = mass;
  out[7] = msum;
  out[8] = umax;
  out[9] = vmax;
  out[10] = wmax;
  out[11] = bad;
  out[12] = sRaoPr * sqrt(rms);
  free(rho); free(ux); free(uy); free(uz); free(T);
}

void oracle_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int oracle_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
