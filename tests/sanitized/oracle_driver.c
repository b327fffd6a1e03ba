/* Drives the CPU oracle through every equation family, limiter mode and
 * boundary kind on small meshes, with every trace array requested, so that
 * an AddressSanitizer / UndefinedBehaviorSanitizer build of the oracle can
 * check its memory accesses and arithmetic.  Exits non-zero on any error
 * the oracle reports or on a non-finite or non-physical result. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "idp_ref.h"

static double frand(unsigned* s) {
  *s = *s * 1103515245u + 12345u;
  return ((*s >> 8) & 0xffff) / 65535.0;
}

/* a discontinuous initial state: quadrant data for Euler, a step plus a
 * sine for the scalar laws */
static void init(const idp_ref_desc* d, double* u, unsigned seed) {
  const long nn = idp_ref_num_nodes(d);
  const int nc = idp_ref_num_comp(d);
  const int n1 = d->p + 1, np = d->dim == 2 ? n1 * n1 : n1;
  for (long i = 0; i < nn; ++i) {
    const long e = i / np;
    const int ex = (int)(e % d->nx), ey = (int)(e / d->nx);
    const double xc = (ex + 0.5) / d->nx, yc = (ey + 0.5) / d->ny;
    const int q = (xc > 0.5) + 2 * (d->dim == 2 && yc > 0.5);
    if (d->eq == IDP_REF_EULER) {
      const double rho = (0.2 + 0.3 * q) * (1.0 + 0.01 * (2.0 * frand(&seed) - 1.0));
      const double vx = 0.3 * (q & 1 ? -1 : 1), vy = d->dim == 2 ? 0.2 * (q & 2 ? -1 : 1) : 0.0;
      const double pr = 0.4 + 0.25 * q;
      u[i] = rho;
      u[nn + i] = rho * vx;
      if (d->dim == 2) u[2 * nn + i] = rho * vy;
      u[(nc - 1) * nn + i] = pr / (d->gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy);
    } else {
      u[i] = 0.5 + 0.5 * sin(6.283185307179586 * xc) + (q ? 0.5 : 0.0) + 0.05 * frand(&seed);
    }
  }
}

static int run(const idp_ref_desc* d, const char* what) {
  const long nn = idp_ref_num_nodes(d);
  const int nc = idp_ref_num_comp(d);
  double* u = calloc((size_t)(nc * nn), sizeof(double));
  double* out = calloc((size_t)(nc * nn), sizeof(double));
  double* trace[10];
  for (int k = 0; k < 10; ++k) trace[k] = calloc((size_t)(nc * nn * (d->dim + 1) + 1), sizeof(double));
  idp_ref_trace tr = {trace[0], trace[1], trace[2], trace[3], trace[4],
                      trace[5], trace[6], trace[7], trace[8], trace[9]};
  int rc = 0;
  init(d, u, 7u);
  double dt = 0.0;
  if (idp_ref_max_dt(d, u, &dt) || !(dt > 0.0)) rc = 1;
  if (!rc && idp_ref_fe(d, u, out, 0.5 * dt, &tr)) rc = 2;
  for (int s = 0; !rc && s < 3; ++s) {
    if (idp_ref_max_dt(d, u, &dt)) rc = 3;
    else if (idp_ref_step(d, u, 0.5 * dt)) rc = 4;
  }
  for (long i = 0; !rc && i < nc * nn; ++i)
    if (!isfinite(u[i])) rc = 5;
  if (!rc && d->eq == IDP_REF_EULER)
    for (long i = 0; i < nn; ++i)
      if (!(u[i] > 0.0)) rc = 6;
  printf("%-36s nodes %6ld  dt %.3e  %s\n", what, nn, dt, rc ? "FAIL" : "ok");
  free(u);
  free(out);
  for (int k = 0; k < 10; ++k) free(trace[k]);
  return rc;
}

int main(void) {
  int bad = 0;
  idp_ref_set_threads(2);
  static const char* lim_name[] = {"subcell", "target", "low", "subcell+si", "elementwise"};
  for (int eq = 0; eq <= 2; ++eq) {
    for (int dim = 1; dim <= 2; ++dim) {
      for (int lim = 0; lim <= 4; ++lim) {
        for (int p = 1; p <= 5; p += 2) {
          idp_ref_desc d;
          memset(&d, 0, sizeof(d));
          d.dim = dim;
          d.nx = 5;
          d.ny = dim == 2 ? 4 : 1;
          d.lx = 1.0;
          d.ly = 1.0;
          d.p = p;
          d.eq = eq;
          d.vel[0] = 1.0;
          d.vel[1] = 0.5;
          d.gamma = 1.4;
          d.limiter = lim;
          d.gmin = 0.0;
          d.gmax = 2.5;
          char what[96];
          snprintf(what, sizeof(what), "eq %d dim %d p %d %s", eq, dim, p, lim_name[lim]);
          bad |= run(&d, what);
        }
      }
    }
  }
  /* open boundaries: prescribed states, outflow and slip walls (Euler) */
  for (int dim = 1; dim <= 2; ++dim) {
    idp_ref_desc d;
    memset(&d, 0, sizeof(d));
    d.dim = dim;
    d.nx = 6;
    d.ny = dim == 2 ? 5 : 1;
    d.lx = 1.0;
    d.ly = 1.0;
    d.p = 3;
    d.eq = IDP_REF_EULER;
    d.gamma = 1.4;
    d.bc[0] = 1;
    d.bc[1] = dim == 2;
    const int n1 = d.p + 1;
    const int nside[4] = {dim == 2 ? d.ny * n1 : 1, dim == 2 ? d.ny * n1 : 1, d.nx * n1, d.nx * n1};
    signed char* types[4];
    double* states[4];
    for (int s = 0; s < 4; ++s) {
      types[s] = malloc((size_t)nside[s]);
      states[s] = malloc(sizeof(double) * (size_t)(nside[s] * (dim + 2)));
      for (int q = 0; q < nside[s]; ++q) {
        types[s][q] = (signed char)(1 + (q + s) % 3);
        states[s][q] = 1.0;
        states[s][nside[s] + q] = 0.1;
        if (dim == 2) states[s][2 * nside[s] + q] = 0.0;
        states[s][(dim + 1) * nside[s] + q] = 2.5;
      }
      d.bc_type[s] = types[s];
      d.bc_state[s] = states[s];
    }
    bad |= run(&d, dim == 2 ? "euler 2-d open sides" : "euler 1-d open sides");
    for (int s = 0; s < 4; ++s) {
      free(types[s]);
      free(states[s]);
    }
  }
  return bad;
}
