/* FP64 CPU oracle of the improved two-component pseudopotential LBM
 * (Sedahmed, Coelho & Warda, arXiv:2111.08666, Sec. 2, Eqs. 1-28).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product path never
 * does.  It shares no code with the HIP implementation.
 *
 * State between steps is the post-collision field f*^s_i(x) (FP64, fluid
 * nodes).  One step = stream with half-way bounce-back, apply the inlet /
 * outlet treatment, then moments, virtual solid density, interaction force and
 * the forced collision.  Observables at time t are taken on the streamed and
 * boundary-completed field f(t).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t q;                /* 9 (D2Q9) or 19 (D3Q19) */
  int32_t nx, ny, nz;       /* nz = 1 for D2Q9 */
  int32_t periodic;         /* bit0 x, bit1 y, bit2 z */
  int32_t open_x;           /* 1: pressure inlet at x = 0, outlet at x = nx-1 */
  int32_t porous_x0, porous_x1; /* saturation window [x0, x1) */
  int32_t bc_set;           /* 3: Set-3 (Sec. 2.3); 1, 2: Set-1, Set-2 */
  int32_t collision;        /* 0 SRT (Eq. 1), 1 MRT, 2 TRT */
  int32_t half_force_shift; /* 1: u = (j + F/2)/rho; 0: u = j/rho */
  int32_t mrt_sj_mode;      /* MRT s_j: 0 min(s_nu, s_q); 1 s_q; 2 s_nu */
  double tau[2];            /* tau^(1), tau^(2) */
  double G;                 /* G_coh = G_ads (Sec. 2.2) */
  double xi;                /* chi1 = 1 + xi, chi2 = 1 - xi */
  double rho_in1, rho_out2; /* Zou-He densities (Eqs. 18-25) */
  double rho_in2, rho_out1; /* Set-1 only */
  double g[3];              /* body acceleration: F^b = rho^s g */
  double lambda;            /* magic parameter (1/s+ - 1/2)(1/s- - 1/2); <= 0: s- = s+ */
  double s_e, s_eps;        /* MRT energy-mode rates; <= 0: equal to s_nu */
  int32_t eq26_mode;        /* reading of Eqs. 26-27: 0 the links hold their initial
                               values; 1 they take the node's own post-collision
                               values (the rule Eq. 28 states for Set-3's inlet) */
  int32_t ivsd_frozen;      /* reading of Eq. 17: 0 the virtual solid density follows
                               the current fluid densities every step; 1 it is
                               evaluated once, on the initial densities, and kept */
} ora_params;

typedef struct {
  int64_t step;
  double mass[2];           /* sum of rho^s over fluid nodes */
  double n_fluid;
  double n_window;          /* fluid nodes in the saturation window */
  double sw_count;          /* window nodes with rho2 > rho1 */
  double sum_rho_w, sum_rho;/* window sums of rho2 and rho1 + rho2 */
  double s_w, s_w_weighted;
  double p_in, p_out, pc;   /* face-averaged EOS pressure (Eq. 14), pc = p_in - p_out */
  double n_in, n_out;
  double flux_in[2];        /* sum of boundary-set populations in the last streaming */
  double flux_out[2];       /* sum of post-collision populations that left the domain */
  int32_t flags;            /* bit0 non-finite density, bit1 negative density */
  int32_t pad;
  double stag[3];           /* staggered momentum: sum over fluid nodes of (-1)^x j_x
                               (resp. y, z) over the total mass, j the momentum of both
                               components' streamed populations */
} ora_obs;

typedef struct ora_sim ora_sim;

/* lattice tables: e (q x 3 ints), w (q doubles), opposite index (q ints) */
int ora_lattice(int q, int32_t *e, double *w, int32_t *opp);

/* Building blocks (exposed for pin tests). u, F are 3-vectors. */
void ora_equilibrium(int q, double rho, const double *u, double *feq);
void ora_forcing(int q, const double *u, const double *F, double *S);   /* Eq. 11 */
/* One-node collision of both components.  fin: 2*q, F: 2*3 (force per
 * component), out: 2*q.  tau_s and u follow Eqs. 5-9 under the readings
 * stated in the source. */
void ora_collide_node(const ora_params *p, const double *fin, const double *F, double *out);
/* The MRT moment matrix (q x q, row-major): the Lallemand-Luo basis for
 * D2Q9, the d'Humieres basis for D3Q19. */
void ora_mrt_matrix(int q, double *M);
/* Zou-He / on-site pressure completion of the links pointing into the domain
 * at an x-face: normal = +1 (inlet, x = 0) or -1 (outlet).  f has q entries;
 * the missing ones are overwritten. */
void ora_zouhe(int q, double *f, double rho_bc, int normal);

/* Simulation.  solid: nx*ny*nz bytes (x fastest), rho0: 2*N initial densities.
 * Returns NULL and writes a message to err (if non-NULL, 256 bytes) on invalid
 * input. */
ora_sim *ora_create(const ora_params *p, const uint8_t *solid, const double *rho0, char *err);
void ora_destroy(ora_sim *s);
void ora_step(ora_sim *s, int64_t n);
void ora_set_bc(ora_sim *s, double rho_in1, double rho_out2);
int64_t ora_get_step(const ora_sim *s);
/* densities at the current time (streamed + boundary-completed field); 2*N */
void ora_density(ora_sim *s, double *rho);
/* interaction + body force per component at the current time; 2*3*N */
void ora_force(ora_sim *s, double *F);
/* pseudopotential field Psi (rho at fluid nodes, virtual density at solid); 2*N */
void ora_psi(ora_sim *s, double *psi);
/* post-collision populations f*[s][i][node] currently held; 2*q*N */
void ora_get_fstar(const ora_sim *s, double *out);
void ora_set_fstar(ora_sim *s, const double *in);
void ora_observables(ora_sim *s, ora_obs *o);
int ora_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
