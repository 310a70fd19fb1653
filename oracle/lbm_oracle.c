/* FP64 CPU oracle of the improved two-component pseudopotential LBM of
 * Sedahmed, Coelho & Warda (arXiv:2111.08666).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no
 * code, header, table or helper with the HIP implementation.
 *
 * Plain and slow on purpose: one loop per step of the method, in the order
 *   stream (with half-way bounce-back, Sec. 2.3)
 *   -> inlet/outlet completion (Set-3, Sec. 2.3, Eqs. 18-28)
 *   -> moments (Eqs. 3, 5)
 *   -> solid pseudopotential (IVSD, Sec. 2.2, Eqs. 16-17)
 *   -> interaction force (Eqs. 12, 13, 15, with the open-boundary mirror of
 *      Sec. 2.1)
 *   -> forced collision (Eqs. 1, 2, 6-11).
 * Readings of points the paper leaves open are marked READING.
 *
 * Parity pins: lattice moments, equilibrium and forcing moments, collision
 * invariants, MRT/TRT/SRT reductions, Zou-He identities, Poiseuille flow,
 * the Laplace law, the flat-interface dissolved density, contact-angle
 * symmetry and the paper's calibration pairs, exact mass bookkeeping.
 * The outlet rule of Eq. 26 (frozen reading), the boundary-pressure window
 * and the saturations are pinned by constructed states with closed-form
 * answers; the pressure form of Eq. 14 (READING below: the pair sum over
 * ordered pairs) by the hydrostatic balance of a mixture at rest under a
 * body force.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Lattices                                                                  */
/* ------------------------------------------------------------------------ */
/* D2Q9 in the paper's order (Sec. 2.1, the e_i matrix and w_i under Eq. 2). */
static const int E9[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},
                             {-1, 0, 0}, {0, -1, 0}, {1, 1, 0},
                             {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* D3Q19 (standard weights 1/3, 1/18, 1/36); the paper's 3D outlook (Sec. 5). */
static const int E19[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double w19(int i) {
  if (i == 0) return 1.0 / 3.0;
  if (i <= 6) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

typedef struct {
  int q;
  int e[19][3];
  double w[19];
  int opp[19];
} lattice;

static int make_lattice(int q, lattice *L) {
  if (q != 9 && q != 19) return -1;
  L->q = q;
  for (int i = 0; i < q; ++i) {
    for (int d = 0; d < 3; ++d) L->e[i][d] = (q == 9) ? E9[i][d] : E19[i][d];
    L->w[i] = (q == 9) ? W9[i] : w19(i);
  }
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j)
      if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] &&
          L->e[j][2] == -L->e[i][2])
        L->opp[i] = j;
  return 0;
}

int ora_lattice(int q, int32_t *e, double *w, int32_t *opp) {
  lattice L;
  if (make_lattice(q, &L)) return -1;
  for (int i = 0; i < q; ++i) {
    for (int d = 0; d < 3; ++d) e[3 * i + d] = L.e[i][d];
    w[i] = L.w[i];
    opp[i] = L.opp[i];
  }
  return 0;
}

static const double CS2 = 1.0 / 3.0; /* c_s^2 with dx = dt = 1 (Sec. 2.1) */

/* Eq. 2: second-order equilibrium at velocity u. */
static void equilibrium(const lattice *L, double rho, const double *u, double *feq) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < L->q; ++i) {
    double eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
    feq[i] = L->w[i] * rho *
             (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* Eq. 11: S_i = w_i [ (e_i - u)/c_s^2 + (e_i.u) e_i / c_s^4 ] . F */
static void forcing(const lattice *L, const double *u, const double *F, double *S) {
  for (int i = 0; i < L->q; ++i) {
    double eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
    double s = 0.0;
    for (int d = 0; d < 3; ++d)
      s += ((L->e[i][d] - u[d]) / CS2 + eu * L->e[i][d] / (CS2 * CS2)) * F[d];
    S[i] = L->w[i] * s;
  }
}

void ora_equilibrium(int q, double rho, const double *u, double *feq) {
  lattice L;
  if (make_lattice(q, &L)) return;
  equilibrium(&L, rho, u, feq);
}

void ora_forcing(int q, const double *u, const double *F, double *S) {
  lattice L;
  if (make_lattice(q, &L)) return;
  forcing(&L, u, F, S);
}

/* ------------------------------------------------------------------------ */
/* D2Q9 moment basis for the MRT-style collision.                            */
/* READING: the paper's collision is SRT; it names MRT only as the route to  */
/* larger viscosity ratios.  The MRT variant uses the Lallemand-Luo D2Q9     */
/* basis (rho, e, eps, jx, qx, jy, qy, pxx, pxy) with the shear rate s_nu =  */
/* 1/tau_s(x), so the viscosity law of Eqs. 6-7 is kept, and the energy-flux */
/* rate s_q from the magic parameter (1/s_nu - 1/2)(1/s_q - 1/2) = lambda.   */
/* ------------------------------------------------------------------------ */
static void mrt_matrix(const lattice *L, double M[9][9], double Minv[9][9]) {
  for (int i = 0; i < 9; ++i) {
    double ex = L->e[i][0], ey = L->e[i][1];
    double e2 = ex * ex + ey * ey;
    M[0][i] = 1.0;
    M[1][i] = -4.0 + 3.0 * e2;
    M[2][i] = 4.0 - 10.5 * e2 + 4.5 * e2 * e2;
    M[3][i] = ex;
    M[4][i] = (-5.0 + 3.0 * e2) * ex;
    M[5][i] = ey;
    M[6][i] = (-5.0 + 3.0 * e2) * ey;
    M[7][i] = ex * ex - ey * ey;
    M[8][i] = ex * ey;
  }
  /* rows are mutually orthogonal, so M^-1 = M^T diag(1/|row|^2) */
  for (int k = 0; k < 9; ++k) {
    double n2 = 0.0;
    for (int i = 0; i < 9; ++i) n2 += M[k][i] * M[k][i];
    for (int i = 0; i < 9; ++i) Minv[i][k] = M[k][i] / n2;
  }
}

/* D3Q19 moment basis of d'Humieres, Ginzburg, Krafczyk, Lallemand & Luo
 * (2002), rows as polynomials of the link vector c (c2 = |c|^2): rho,
 * e = 19 c2 - 30, eps = (21 c2^2 - 53 c2 + 24)/2, j and q = (5 c2 - 9) c per
 * axis, 3 p_xx = 3 cx^2 - c2 and pi_xx = (3 c2 - 5)(3 cx^2 - c2),
 * p_ww = cy^2 - cz^2 and pi_ww = (3 c2 - 5)(cy^2 - cz^2), p_xy, p_yz, p_xz,
 * and the third-order m_x = (cy^2 - cz^2) cx, m_y = (cz^2 - cx^2) cy,
 * m_z = (cx^2 - cy^2) cz.  Row order: rho, e, eps, jx, qx, jy, qy, jz, qz,
 * 3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz. */
static void mrt_matrix19(const lattice *L, double M[19][19], double Minv[19][19]) {
  for (int i = 0; i < 19; ++i) {
    double cx = L->e[i][0], cy = L->e[i][1], cz = L->e[i][2];
    double c2 = cx * cx + cy * cy + cz * cz;
    M[0][i] = 1.0;
    M[1][i] = 19.0 * c2 - 30.0;
    M[2][i] = (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    M[3][i] = cx;
    M[4][i] = (5.0 * c2 - 9.0) * cx;
    M[5][i] = cy;
    M[6][i] = (5.0 * c2 - 9.0) * cy;
    M[7][i] = cz;
    M[8][i] = (5.0 * c2 - 9.0) * cz;
    M[9][i] = 3.0 * cx * cx - c2;
    M[10][i] = (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2);
    M[11][i] = cy * cy - cz * cz;
    M[12][i] = (3.0 * c2 - 5.0) * (cy * cy - cz * cz);
    M[13][i] = cx * cy;
    M[14][i] = cy * cz;
    M[15][i] = cx * cz;
    M[16][i] = (cy * cy - cz * cz) * cx;
    M[17][i] = (cz * cz - cx * cx) * cy;
    M[18][i] = (cx * cx - cy * cy) * cz;
  }
  for (int k = 0; k < 19; ++k) {
    double n2 = 0.0;
    for (int i = 0; i < 19; ++i) n2 += M[k][i] * M[k][i];
    for (int i = 0; i < 19; ++i) Minv[i][k] = M[k][i] / n2;
  }
}

void ora_mrt_matrix(int q, double *M) {
  lattice L;
  if (make_lattice(q, &L)) return;
  if (q == 9) {
    double A[9][9], B[9][9];
    mrt_matrix(&L, A, B);
    for (int k = 0; k < 81; ++k) M[k] = A[k / 9][k % 9];
  } else {
    double A[19][19], B[19][19];
    mrt_matrix19(&L, A, B);
    for (int k = 0; k < 361; ++k) M[k] = A[k / 19][k % 19];
  }
}

/* Relaxation rates at one node.  READING (Eq. 7 as printed has tau + 1/2;
 * the paper's own numbers tau = 3.5 -> nu = 1 and tau = 0.62 -> nu = 0.04
 * need nu = c_s^2 (tau - 1/2)): Eq. 6 then gives tau_s as the
 * density-weighted mean of tau^(1) and tau^(2). */
typedef struct {
  double tau_s, s_nu, s_q, s_e, s_eps, s_j;
} rates;

static rates node_rates(const ora_params *p, double rho1, double rho2) {
  rates r;
  r.tau_s = (rho1 * p->tau[0] + rho2 * p->tau[1]) / (rho1 + rho2);
  r.s_nu = 1.0 / r.tau_s;
  r.s_q = (p->lambda > 0.0) ? 1.0 / (0.5 + p->lambda / (r.tau_s - 0.5)) : r.s_nu;
  r.s_e = (p->s_e > 0.0) ? p->s_e : r.s_nu;
  r.s_eps = (p->s_eps > 0.0) ? p->s_eps : r.s_nu;
  /* component-momentum rate (READING: the paper names MRT but gives no
   * rates): mode 0 the smaller of s_nu and s_q, so that neither end of the
   * viscosity range over-relaxes the components' momenta; 1 s_q; 2 s_nu */
  if (p->mrt_sj_mode == 1) r.s_j = r.s_q;
  else if (p->mrt_sj_mode == 2) r.s_j = r.s_nu;
  else r.s_j = r.s_nu < r.s_q ? r.s_nu : r.s_q;
  return r;
}

/* Forced collision of both components at one node (Eqs. 1-11).
 * READING (Eqs. 4, 8, 9): tau_s is common to both components, so Eq. 8's
 * common velocity is the barycentric one, sum_s j^s / rho; it carries the
 * half-force shift F/2 (switchable) so that Eq. 1's (1 - 1/2tau_s) forcing
 * factor adds exactly F of momentum per step. */
static void collide(const lattice *L, const ora_params *p, const double *fin,
                    const double *F, double *out) {
  const int q = L->q;
  double rho_s[2] = {0.0, 0.0}, j[3] = {0.0, 0.0, 0.0}, Ft[3];
  for (int s = 0; s < 2; ++s)
    for (int i = 0; i < q; ++i) {
      rho_s[s] += fin[s * q + i];
      for (int d = 0; d < 3; ++d) j[d] += L->e[i][d] * fin[s * q + i];
    }
  double rho = rho_s[0] + rho_s[1];
  double h = p->half_force_shift ? 0.5 : 0.0;
  double u[3];
  for (int d = 0; d < 3; ++d) {
    Ft[d] = F[d] + F[3 + d];
    u[d] = (j[d] + h * Ft[d]) / rho;
  }
  rates r = node_rates(p, rho_s[0], rho_s[1]);

  for (int s = 0; s < 2; ++s) {
    const double *f = fin + s * q;
    double feq[19], S[19];
    equilibrium(L, rho_s[s], u, feq);
    forcing(L, u, F + 3 * s, S);
    double *o = out + s * q;
    if (p->collision == 0) { /* SRT, Eq. 1 */
      for (int i = 0; i < q; ++i)
        o[i] = f[i] - (f[i] - feq[i]) / r.tau_s + (1.0 - 1.0 / (2.0 * r.tau_s)) * S[i];
    } else if (p->collision == 1) { /* MRT in moment space */
      double M[19][19], Mi[19][19]; /* the leading q x q block is used */
      double sr[19];
      if (q == 9) {
        double A[9][9], B[9][9];
        mrt_matrix(L, A, B);
        for (int k = 0; k < 9; ++k)
          for (int i = 0; i < 9; ++i) { M[k][i] = A[k][i]; Mi[k][i] = B[k][i]; }
        const double s9[9] = {1.0, r.s_e, r.s_eps, r.s_j, r.s_q, r.s_j, r.s_q, r.s_nu, r.s_nu};
        for (int k = 0; k < 9; ++k) sr[k] = s9[k];
      } else {
        mrt_matrix19(L, M, Mi);
        /* READING: the paper gives no rates.  The second-order moments relax
         * at s_nu (viscosity of Eqs. 6-7), e and eps at the free energy rates,
         * the fourth-order pi moments at s_eps and the third-order m moments
         * at s_q, so that equal even and odd rates give TRT and equal rates
         * give SRT. */
        const double s19[19] = {1.0,    r.s_e,  r.s_eps, r.s_j,  r.s_q,  r.s_j,  r.s_q,
                                r.s_j,  r.s_q,  r.s_nu,  r.s_eps, r.s_nu, r.s_eps, r.s_nu,
                                r.s_nu, r.s_nu, r.s_q,   r.s_q,  r.s_q};
        for (int k = 0; k < 19; ++k) sr[k] = s19[k];
      }
      double mstar[19];
      for (int k = 0; k < q; ++k) {
        double m = 0.0, meq = 0.0, ms = 0.0;
        for (int i = 0; i < q; ++i) {
          m += M[k][i] * f[i];
          meq += M[k][i] * feq[i];
          ms += M[k][i] * S[i];
        }
        mstar[k] = m - sr[k] * (m - meq) + (1.0 - 0.5 * sr[k]) * ms;
      }
      for (int i = 0; i < q; ++i) {
        double v = 0.0;
        for (int k = 0; k < q; ++k) v += Mi[i][k] * mstar[k];
        o[i] = v;
      }
    } else { /* TRT: symmetric part at s+ = s_nu, antisymmetric at s- = s_q */
      double sp = r.s_nu, sm = r.s_q;
      for (int i = 0; i < q; ++i) {
        int b = L->opp[i];
        double fp = 0.5 * (f[i] + f[b]), fm = 0.5 * (f[i] - f[b]);
        double ep = 0.5 * (feq[i] + feq[b]), em = 0.5 * (feq[i] - feq[b]);
        double Sp = 0.5 * (S[i] + S[b]), Sm = 0.5 * (S[i] - S[b]);
        o[i] = f[i] - sp * (fp - ep) - sm * (fm - em) + (1.0 - 0.5 * sp) * Sp +
               (1.0 - 0.5 * sm) * Sm;
      }
    }
  }
}

void ora_collide_node(const ora_params *p, const double *fin, const double *F, double *out) {
  lattice L;
  if (make_lattice(p->q, &L)) return;
  collide(&L, p, fin, F, out);
}

/* ------------------------------------------------------------------------ */
/* Zou-He pressure completion (Eqs. 18-25; Zou & He 1997).                   */
/* With m = rho_bc - sum(parallel) - 2 sum(outgoing) the normal mass flux,   */
/* a missing population takes f_i = f_opp(i) + 6 w_i m - e_i,t . N_t, where  */
/* N_t is half the tangential momentum of the known parallel links.  For     */
/* D2Q9 this is Eqs. 19-21 and 23-25 term by term; for D3Q19 it is the       */
/* on-site construction of Hecht & Harting (2010) with zero tangential       */
/* velocity.                                                                 */
/* ------------------------------------------------------------------------ */
static void zouhe(const lattice *L, double *f, double rho_bc, int normal) {
  double par = 0.0, outg = 0.0, Nt[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < L->q; ++i) {
    int ex = L->e[i][0];
    if (ex == 0) {
      par += f[i];
      Nt[1] += 0.5 * L->e[i][1] * f[i];
      Nt[2] += 0.5 * L->e[i][2] * f[i];
    } else if (ex == -normal) {
      outg += f[i];
    }
  }
  double m = rho_bc - par - 2.0 * outg; /* = normal * rho_bc * u_x */
  for (int i = 0; i < L->q; ++i) {
    if (L->e[i][0] != normal) continue;
    f[i] = f[L->opp[i]] + 6.0 * L->w[i] * m - L->e[i][1] * Nt[1] - L->e[i][2] * Nt[2];
  }
}

void ora_zouhe(int q, double *f, double rho_bc, int normal) {
  lattice L;
  if (make_lattice(q, &L)) return;
  zouhe(&L, f, rho_bc, normal);
}

/* ------------------------------------------------------------------------ */
/* Simulation                                                                */
/* ------------------------------------------------------------------------ */
struct ora_sim {
  ora_params p;
  lattice L;
  int nx, ny, nz;
  int64_t N;
  uint8_t *solid;
  double *fs;     /* post-collision f*, [2][q][N] */
  double *f;      /* streamed + completed f, [2][q][N] */
  double *rho;    /* [2][N] */
  double *psi;    /* [2][N] */
  double *F;      /* [2][3][N] */
  double *frozen; /* [2][q][ny*nz]: [0] comp-1 at outlet, [1] comp-2 at inlet */
  double *psi0;   /* [2][N]: Eq. 17 on the initial densities (ivsd_frozen) */
  double flux_in[2], flux_out[2];
  int64_t step;
};

#define FS(s, c, i, n) ((s)->fs[((int64_t)(c) * (s)->L.q + (i)) * (s)->N + (n)])
#define FF(s, c, i, n) ((s)->f[((int64_t)(c) * (s)->L.q + (i)) * (s)->N + (n)])
#define RHO(s, c, n) ((s)->rho[(int64_t)(c) * (s)->N + (n)])
#define PSI(s, c, n) ((s)->psi[(int64_t)(c) * (s)->N + (n)])
#define FRC(s, c, d, n) ((s)->F[((int64_t)(c) * 3 + (d)) * (s)->N + (n)])
#define FRZ(s, c, i, t) ((s)->frozen[((int64_t)(c) * (s)->L.q + (i)) * ((int64_t)(s)->ny * (s)->nz) + (t)])

static int64_t idx3(const ora_sim *s, int x, int y, int z) {
  return (int64_t)x + (int64_t)s->nx * ((int64_t)y + (int64_t)s->ny * z);
}

/* Neighbour coordinate along one axis: wraps on periodic axes.  Returns 0 if
 * inside the domain, 1 if it leaves the domain. */
static int wrap1(int *c, int n, int periodic) {
  if (*c >= 0 && *c < n) return 0;
  if (periodic) {
    *c = ((*c % n) + n) % n;
    return 0;
  }
  return 1;
}

/* Node at x + d.  Returns 0 inside (nb set), 1 if it leaves across the open
 * x faces, 2 if it leaves across any other closed edge. */
static int neighbor(const ora_sim *s, int x, int y, int z, int dx, int dy, int dz,
                    int64_t *nb) {
  int a = x + dx, b = y + dy, c = z + dz;
  int ox = wrap1(&a, s->nx, s->p.periodic & 1);
  int oy = wrap1(&b, s->ny, s->p.periodic & 2);
  int oz = wrap1(&c, s->nz, s->p.periodic & 4);
  if (oy || oz) return 2;
  if (ox) return s->p.open_x ? 1 : 2;
  *nb = idx3(s, a, b, c);
  return 0;
}

static void coords(const ora_sim *s, int64_t n, int *x, int *y, int *z) {
  *x = (int)(n % s->nx);
  *y = (int)((n / s->nx) % s->ny);
  *z = (int)(n / ((int64_t)s->nx * s->ny));
}

static void set_err(char *err, const char *msg) {
  if (err) snprintf(err, 256, "%s", msg);
}

static void solid_psi(const ora_sim *s, int64_t n, const double *rho, double *psi1, double *psi2);

ora_sim *ora_create(const ora_params *p, const uint8_t *solid, const double *rho0, char *err) {
  lattice L;
  if (make_lattice(p->q, &L)) { set_err(err, "q must be 9 or 19"); return NULL; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) { set_err(err, "bad grid size"); return NULL; }
  if (p->q == 9 && p->nz != 1) { set_err(err, "D2Q9 needs nz = 1"); return NULL; }
  if (p->open_x && ((p->periodic & 1) || p->nx < 3)) {
    set_err(err, "open x needs nx >= 3 and x not periodic"); return NULL;
  }
  for (int c = 0; c < 2; ++c)
    if (!(p->tau[c] > 0.5) || !isfinite(p->tau[c])) { set_err(err, "tau must exceed 1/2"); return NULL; }
  if (!(fabs(p->xi) < 1.0)) { set_err(err, "|xi| must be < 1"); return NULL; }
  if (p->collision < 0 || p->collision > 2) {
    set_err(err, "collision: 0 SRT, 1 MRT, 2 TRT"); return NULL;
  }
  if (p->bc_set < 1 || p->bc_set > 3) { set_err(err, "bc_set must be 1, 2 or 3"); return NULL; }
  if (p->eq26_mode != 0 && p->eq26_mode != 1) { set_err(err, "eq26_mode must be 0 or 1"); return NULL; }
  if (p->ivsd_frozen != 0 && p->ivsd_frozen != 1) { set_err(err, "ivsd_frozen must be 0 or 1"); return NULL; }

  ora_sim *s = (ora_sim *)calloc(1, sizeof(ora_sim));
  s->p = *p;
  s->L = L;
  s->nx = p->nx; s->ny = p->ny; s->nz = p->nz;
  s->N = (int64_t)p->nx * p->ny * p->nz;
  const int q = L.q;
  const int64_t N = s->N;

  /* every fluid node must only reach in-domain nodes except across open x */
  for (int64_t n = 0; n < N; ++n) {
    if (solid[n]) continue;
    int x, y, z, nfl = 0;
    coords(s, n, &x, &y, &z);
    for (int i = 1; i < q; ++i) {
      int64_t nb;
      int r = neighbor(s, x, y, z, L.e[i][0], L.e[i][1], L.e[i][2], &nb);
      if (r == 2) {
        set_err(err, "fluid node touches a closed domain edge (make it solid or periodic)");
        free(s); return NULL;
      }
      if (r == 0 && !solid[nb]) ++nfl;
    }
    if (p->open_x && (x == 0 || x == s->nx - 1) && nfl == 0) {
      set_err(err, "fluid node on an open face without a fluid neighbour");
      free(s); return NULL;
    }
    for (int c = 0; c < 2; ++c) {
      double r0 = rho0[(int64_t)c * N + n];
      if (!isfinite(r0) || r0 < 0.0) { set_err(err, "initial densities must be finite and >= 0"); free(s); return NULL; }
    }
    if (!(rho0[n] + rho0[N + n] > 0.0)) { set_err(err, "total initial density must be > 0"); free(s); return NULL; }
  }

  s->solid = (uint8_t *)malloc((size_t)N);
  memcpy(s->solid, solid, (size_t)N);
  s->fs = (double *)calloc((size_t)(2 * q * N), sizeof(double));
  s->f = (double *)calloc((size_t)(2 * q * N), sizeof(double));
  s->rho = (double *)calloc((size_t)(2 * N), sizeof(double));
  s->psi = (double *)calloc((size_t)(2 * N), sizeof(double));
  s->F = (double *)calloc((size_t)(6 * N), sizeof(double));
  s->frozen = (double *)calloc((size_t)(2 * q * s->ny * s->nz), sizeof(double));
  s->psi0 = (double *)calloc((size_t)(2 * N), sizeof(double));

  /* READING (initial state): the given densities are placed as rest
   * equilibria w_i rho0 in the post-collision field, so the first step
   * starts by streaming them. */
  for (int64_t n = 0; n < N; ++n) {
    if (solid[n]) continue;
    for (int c = 0; c < 2; ++c)
      for (int i = 0; i < q; ++i) FS(s, c, i, n) = L.w[i] * rho0[(int64_t)c * N + n];
  }
  /* Eq. 26 (and Eq. 27 for Set-2): READING "frozen" - the populations that
   * keep themselves never change, so they hold the initial rest equilibrium. */
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y) {
      int t = y + s->ny * z;
      int64_t no = idx3(s, s->nx - 1, y, z), ni = idx3(s, 0, y, z);
      for (int i = 0; i < q; ++i) {
        FRZ(s, 0, i, t) = L.w[i] * rho0[no];
        FRZ(s, 1, i, t) = L.w[i] * rho0[N + ni];
      }
    }
  /* Eq. 17, READING "frozen" (ivsd_frozen = 1): evaluated once, on the
   * initial densities, and used at every step. */
  if (p->ivsd_frozen)
    for (int64_t n = 0; n < N; ++n)
      if (solid[n]) solid_psi(s, n, rho0, &s->psi0[n], &s->psi0[N + n]);
  s->step = 0;
  return s;
}

void ora_destroy(ora_sim *s) {
  if (!s) return;
  free(s->solid); free(s->fs); free(s->f); free(s->rho); free(s->psi);
  free(s->F); free(s->frozen); free(s->psi0); free(s);
}

void ora_set_bc(ora_sim *s, double rho_in1, double rho_out2) {
  s->p.rho_in1 = rho_in1;
  s->p.rho_out2 = rho_out2;
}

int64_t ora_get_step(const ora_sim *s) { return s->step; }

/* Pull streaming with half-way bounce-back: f_i(x) = f*_i(x - e_i), or
 * f*_opp(i)(x) if x - e_i is solid.  Links whose source lies outside across
 * an open face are completed by the inlet/outlet treatment. */
static void stream_complete(ora_sim *s) {
  const lattice *L = &s->L;
  const int q = L->q;
  const int64_t N = s->N;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    if (s->solid[n]) continue;
    int x, y, z;
    coords(s, n, &x, &y, &z);
    for (int c = 0; c < 2; ++c)
      for (int i = 0; i < q; ++i) {
        int64_t src;
        int r = neighbor(s, x, y, z, -L->e[i][0], -L->e[i][1], -L->e[i][2], &src);
        if (r != 0)
          FF(s, c, i, n) = NAN; /* missing: set below */
        else if (s->solid[src])
          FF(s, c, i, n) = FS(s, c, L->opp[i], n);
        else
          FF(s, c, i, n) = FS(s, c, i, src);
      }
  }
  s->flux_in[0] = s->flux_in[1] = s->flux_out[0] = s->flux_out[1] = 0.0;
  if (!s->p.open_x) return;
  const int set = s->p.bc_set;
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y) {
      int t = y + s->ny * z;
      for (int side = 0; side < 2; ++side) {
        int x = side == 0 ? 0 : s->nx - 1;
        int normal = side == 0 ? 1 : -1; /* direction of the missing links */
        int64_t n = idx3(s, x, y, z);
        if (s->solid[n]) continue;
        for (int c = 0; c < 2; ++c) {
          double f[19];
          for (int i = 0; i < q; ++i) f[i] = FF(s, c, i, n);
          /* populations leaving across this face */
          for (int i = 0; i < q; ++i)
            if (L->e[i][0] == -normal) s->flux_out[c] += FS(s, c, i, n);
          int zou; /* does Zou-He set this component here? */
          double rho_bc;
          if (side == 0) { zou = (c == 0) || set == 1; rho_bc = c == 0 ? s->p.rho_in1 : s->p.rho_in2; }
          else { zou = (c == 1) || set == 1; rho_bc = c == 1 ? s->p.rho_out2 : s->p.rho_out1; }
          if (zou) {
            zouhe(L, f, rho_bc, normal);
          } else if (side == 1 || set == 2) {
            /* Eq. 26 (outlet, comp 1) and Eq. 27 (inlet, comp 2, Set-2).
             * READING 0 (default): the links "maintain themselves" through
             * collision and streaming, so they never change from their
             * initial values.  READING 1: they keep the node's own
             * post-collision values, the rule Eq. 28 writes out. */
            int fc = side == 1 ? 0 : 1;
            for (int i = 0; i < q; ++i)
              if (L->e[i][0] == normal) f[i] = s->p.eq26_mode ? FS(s, c, i, n) : FRZ(s, fc, i, t);
          } else {
            /* Eq. 28 (Set-3, inlet, comp 2): keep this node's post-collision value */
            for (int i = 0; i < q; ++i)
              if (L->e[i][0] == normal) f[i] = FS(s, c, i, n);
          }
          for (int i = 0; i < q; ++i) {
            if (L->e[i][0] == normal) s->flux_in[c] += f[i];
            FF(s, c, i, n) = f[i];
          }
        }
      }
    }
}

/* Eqs. 3, 5 */
static void moments(ora_sim *s) {
  const int q = s->L.q;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < s->N; ++n)
    for (int c = 0; c < 2; ++c) {
      double r = 0.0;
      if (!s->solid[n])
        for (int i = 0; i < q; ++i) r += FF(s, c, i, n);
      RHO(s, c, n) = r;
    }
}

/* Eqs. 16-17 (IVSD): at a solid node n the pseudopotential is the virtual
 * density chi^s * (w-weighted mean of rho^s over in-domain fluid neighbours),
 * here of the density field rho ([2][N]).  A solid node with no fluid
 * neighbour gets 0 (it never enters a fluid node's force). */
static void solid_psi(const ora_sim *s, int64_t n, const double *rho, double *psi1, double *psi2) {
  const lattice *L = &s->L;
  const double chi[2] = {1.0 + s->p.xi, 1.0 - s->p.xi};
  int x, y, z;
  coords(s, n, &x, &y, &z);
  double num[2] = {0.0, 0.0}, den = 0.0;
  for (int i = 1; i < L->q; ++i) {
    int64_t nb;
    if (neighbor(s, x, y, z, L->e[i][0], L->e[i][1], L->e[i][2], &nb) != 0) continue;
    if (s->solid[nb]) continue;
    den += L->w[i];
    for (int c = 0; c < 2; ++c) num[c] += L->w[i] * rho[(int64_t)c * s->N + nb];
  }
  *psi1 = den > 0.0 ? chi[0] * num[0] / den : 0.0;
  *psi2 = den > 0.0 ? chi[1] * num[1] / den : 0.0;
}

/* The pseudopotential field: psi = rho at fluid nodes (Sec. 2.1); at solid
 * nodes Eq. 17, READING: recomputed every step from the current densities
 * (default), or the values Eq. 17 gave on the initial densities
 * (ivsd_frozen). */
static void pseudopotential(ora_sim *s) {
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < s->N; ++n) {
    if (!s->solid[n]) {
      for (int c = 0; c < 2; ++c) PSI(s, c, n) = RHO(s, c, n);
    } else if (s->p.ivsd_frozen) {
      for (int c = 0; c < 2; ++c) PSI(s, c, n) = s->psi0[(int64_t)c * s->N + n];
    } else {
      solid_psi(s, n, s->rho, &PSI(s, 0, n), &PSI(s, 1, n));
    }
  }
}

/* Eqs. 12, 13, 15 with G_ads = G_coh: F^s = -G rho^s sum_i w_i Psi^sbar(x+e_i) e_i
 * + rho^s g.  Across an open x face the missing neighbour is replaced by the
 * opposite one, x - e_i (Sec. 2.1, the mirror rule for boundary points). */
static void force(ora_sim *s) {
  const lattice *L = &s->L;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < s->N; ++n) {
    for (int c = 0; c < 2; ++c)
      for (int d = 0; d < 3; ++d) FRC(s, c, d, n) = 0.0;
    if (s->solid[n]) continue;
    int x, y, z;
    coords(s, n, &x, &y, &z);
    for (int c = 0; c < 2; ++c) {
      int cb = 1 - c;
      double sum[3] = {0.0, 0.0, 0.0};
      for (int i = 1; i < L->q; ++i) {
        int64_t nb;
        int r = neighbor(s, x, y, z, L->e[i][0], L->e[i][1], L->e[i][2], &nb);
        if (r == 1) neighbor(s, x, y, z, -L->e[i][0], -L->e[i][1], -L->e[i][2], &nb);
        for (int d = 0; d < 3; ++d) sum[d] += L->w[i] * PSI(s, cb, nb) * L->e[i][d];
      }
      for (int d = 0; d < 3; ++d)
        FRC(s, c, d, n) = -s->p.G * RHO(s, c, n) * sum[d] + RHO(s, c, n) * s->p.g[d];
    }
  }
}

static void collide_all(ora_sim *s) {
  const lattice *L = &s->L;
  const int q = L->q;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < s->N; ++n) {
    if (s->solid[n]) continue;
    double fin[38], F[6], out[38];
    for (int c = 0; c < 2; ++c) {
      for (int i = 0; i < q; ++i) fin[c * q + i] = FF(s, c, i, n);
      for (int d = 0; d < 3; ++d) F[3 * c + d] = FRC(s, c, d, n);
    }
    collide(L, &s->p, fin, F, out);
    for (int c = 0; c < 2; ++c)
      for (int i = 0; i < q; ++i) FS(s, c, i, n) = out[c * q + i];
  }
}

void ora_step(ora_sim *s, int64_t n) {
  for (int64_t k = 0; k < n; ++k) {
    stream_complete(s);
    moments(s);
    pseudopotential(s);
    force(s);
    collide_all(s);
    s->step++;
  }
}

void ora_density(ora_sim *s, double *rho) {
  stream_complete(s);
  moments(s);
  memcpy(rho, s->rho, sizeof(double) * 2 * (size_t)s->N);
}

void ora_psi(ora_sim *s, double *psi) {
  stream_complete(s);
  moments(s);
  pseudopotential(s);
  memcpy(psi, s->psi, sizeof(double) * 2 * (size_t)s->N);
}

void ora_force(ora_sim *s, double *F) {
  stream_complete(s);
  moments(s);
  pseudopotential(s);
  force(s);
  memcpy(F, s->F, sizeof(double) * 6 * (size_t)s->N);
}

void ora_get_fstar(const ora_sim *s, double *out) {
  memcpy(out, s->fs, sizeof(double) * 2 * (size_t)s->L.q * (size_t)s->N);
}

void ora_set_fstar(ora_sim *s, const double *in) {
  memcpy(s->fs, in, sizeof(double) * 2 * (size_t)s->L.q * (size_t)s->N);
}

/* Is this face node at least 3 lattice units from every solid node
 * (Chebyshev distance)?  READING of "ignore the pressure values near the
 * solid walls" (Sec. 2.3). */
static int far_from_solid(const ora_sim *s, int x, int y, int z) {
  int rz = s->nz > 1 ? 2 : 0;
  for (int dz = -rz; dz <= rz; ++dz)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        int64_t nb;
        if (neighbor(s, x, y, z, dx, dy, dz, &nb) != 0) continue;
        if (s->solid[nb]) return 0;
      }
  return 1;
}

/* Observables on f(t).  Pressure: Eq. 14 with the pair sum over ordered
 * pairs s != sbar, P = c_s^2 (rho1 + rho2) + c_s^2 G rho1 rho2 (READING).
 * Water (component 2, wetting) saturation: READING - the count of fluid
 * nodes of the window with rho2 > rho1, over the window's fluid nodes, and a
 * density-weighted variant sum rho2 / sum (rho1 + rho2). */
void ora_observables(ora_sim *s, ora_obs *o) {
  stream_complete(s);
  moments(s);
  memset(o, 0, sizeof(*o));
  o->step = s->step;
  int x0 = s->p.porous_x0, x1 = s->p.porous_x1 > 0 ? s->p.porous_x1 : s->nx;
  double pin = 0.0, pout = 0.0;
  for (int64_t n = 0; n < s->N; ++n) {
    if (s->solid[n]) continue;
    int x, y, z;
    coords(s, n, &x, &y, &z);
    double r1 = RHO(s, 0, n), r2 = RHO(s, 1, n);
    if (!isfinite(r1) || !isfinite(r2)) o->flags |= 1;
    if (r1 < 0.0 || r2 < 0.0) o->flags |= 2;
    o->mass[0] += r1;
    o->mass[1] += r2;
    o->n_fluid += 1.0;
    if (x >= x0 && x < x1) {
      o->n_window += 1.0;
      if (r2 > r1) o->sw_count += 1.0;
      o->sum_rho_w += r2;
      o->sum_rho += r1 + r2;
    }
    if ((x == 0 || x == s->nx - 1) && far_from_solid(s, x, y, z)) {
      double P = CS2 * (r1 + r2) + CS2 * s->p.G * r1 * r2;
      if (x == 0) { pin += P; o->n_in += 1.0; }
      else { pout += P; o->n_out += 1.0; }
    }
    /* momentum of the streamed populations, both components, signed by
       the parity of each coordinate */
    const int xyz[3] = {x, y, z};
    for (int d = 0; d < 3; ++d) {
      double j = 0.0;
      for (int c = 0; c < 2; ++c)
        for (int i = 0; i < s->L.q; ++i) j += s->L.e[i][d] * FF(s, c, i, n);
      o->stag[d] += (xyz[d] & 1) ? -j : j;
    }
  }
  o->s_w = o->n_window > 0 ? o->sw_count / o->n_window : 0.0;
  o->s_w_weighted = o->sum_rho > 0 ? o->sum_rho_w / o->sum_rho : 0.0;
  o->p_in = o->n_in > 0 ? pin / o->n_in : 0.0;
  o->p_out = o->n_out > 0 ? pout / o->n_out : 0.0;
  o->pc = o->p_in - o->p_out;
  const double m = o->mass[0] + o->mass[1];
  for (int d = 0; d < 3; ++d) o->stag[d] = m > 0.0 ? o->stag[d] / m : 0.0;
  for (int c = 0; c < 2; ++c) {
    o->flux_in[c] = s->flux_in[c];
    o->flux_out[c] = s->flux_out[c];
  }
}

int ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
