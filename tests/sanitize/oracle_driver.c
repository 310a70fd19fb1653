/* Sanitizer driver for the FP64 oracle (test infrastructure): runs small
 * D2Q9 and D3Q19 cases through every boundary set, both readings of
 * Eqs. 26-27 and of Eq. 17 and every collision operator, and every read-out,
 * so that an
 * AddressSanitizer / UndefinedBehaviorSanitizer build sees each code path.
 * Exits 0 when every run stays finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/lbm_oracle.h"

static unsigned rnd(unsigned *s) { *s = *s * 1103515245u + 12345u; return (*s >> 16) & 0x7fffu; }

static int run_case(int q, int nx, int ny, int nz, int open_x, int bc_set, int eq26, int coll, unsigned seed,
                    int ivsd_frozen) {
  const int N = nx * ny * nz;
  uint8_t *solid = calloc((size_t)N, 1);
  double *rho0 = calloc((size_t)2 * N, sizeof(double));
  unsigned s = seed;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int n = x + nx * (y + ny * z);
        const int wall = y == 0 || y == ny - 1 || (q == 19 && (z == 0 || z == nz - 1));
        const int interior = x > 3 && x < nx - 4;
        /* open boxes: walls and random obstacles; periodic boxes: all fluid */
        solid[n] = (uint8_t)(open_x && (wall || (interior && rnd(&s) % 9 == 0)));
        const int inv = open_x ? x < 4 : (x - nx / 2) * (x - nx / 2) + (y - ny / 2) * (y - ny / 2) < 16;
        rho0[n] = solid[n] ? 0.0 : (inv ? 1.0 : 0.027);
        rho0[N + n] = solid[n] ? 0.0 : (inv ? 0.027 : 1.0);
      }
  ora_params p = {0};
  p.q = q; p.nx = nx; p.ny = ny; p.nz = nz;
  p.periodic = open_x ? 0 : (q == 19 ? 7 : 3);
  p.open_x = open_x; p.porous_x0 = 4; p.porous_x1 = nx - 4;
  p.bc_set = bc_set; p.collision = coll; p.half_force_shift = 1; p.mrt_sj_mode = 0;
  p.tau[0] = 1.7; p.tau[1] = 0.62; p.G = 3.5; p.xi = -0.3;
  p.rho_in1 = 1.02; p.rho_out2 = 1.0; p.rho_in2 = 0.027; p.rho_out1 = 0.027;
  p.lambda = 3.0 / 16.0; p.s_e = 1.0; p.s_eps = 1.0; p.eq26_mode = eq26; p.ivsd_frozen = ivsd_frozen;
  char err[256];
  ora_sim *sim = ora_create(&p, solid, rho0, err);
  if (!sim) {
    fprintf(stderr, "create failed: %s\n", err);
    free(solid); free(rho0);
    return 1;
  }
  ora_step(sim, 25);
  ora_set_bc(sim, 1.03, 0.99);
  ora_step(sim, 5);
  double *rho = malloc(sizeof(double) * 2 * N), *psi = malloc(sizeof(double) * 2 * N);
  double *F = malloc(sizeof(double) * 6 * N), *fs = malloc(sizeof(double) * 2 * q * N);
  ora_density(sim, rho);
  ora_psi(sim, psi);
  ora_force(sim, F);
  ora_get_fstar(sim, fs);
  ora_set_fstar(sim, fs);
  ora_obs o;
  ora_observables(sim, &o);
  int bad = o.flags & 1;
  for (int n = 0; n < 2 * N; ++n) bad |= !isfinite(rho[n]);
  free(rho); free(psi); free(F); free(fs);
  ora_destroy(sim);
  free(solid); free(rho0);
  if (bad) fprintf(stderr, "non-finite: q %d set %d eq26 %d coll %d\n", q, bc_set, eq26, coll);
  return bad;
}

int main(void) {
  int fails = 0;
  for (int coll = 0; coll < 3; ++coll)
    for (int set = 1; set <= 3; ++set)
      for (int eq26 = 0; eq26 < 2; ++eq26) fails += run_case(9, 40, 18, 1, 1, set, eq26, coll, 7u + set, eq26);
  fails += run_case(9, 24, 20, 1, 0, 3, 0, 2, 3u, 0);
  for (int coll = 0; coll < 3; ++coll) fails += run_case(19, 20, 12, 10, 1, 3, coll == 1, coll, 11u, coll == 2);
  fails += run_case(19, 12, 10, 8, 0, 3, 0, 2, 5u, 1);
  /* building blocks */
  int32_t e[57], opp[19];
  double w[19], feq[19], S[19], u[3] = {0.02, -0.01, 0.005}, Fv[3] = {1e-4, 0, -2e-4};
  double M[361], f[19];
  for (int q = 9; q <= 19; q += 10) {
    ora_lattice(q, e, w, opp);
    ora_equilibrium(q, 1.0, u, feq);
    ora_forcing(q, u, Fv, S);
    ora_mrt_matrix(q, M);
    for (int i = 0; i < q; ++i) f[i] = feq[i];
    ora_zouhe(q, f, 1.01, 1);
    ora_zouhe(q, f, 0.99, -1);
  }
  printf("oracle sanitizer driver: %d failing cases\n", fails);
  return fails != 0;
}
