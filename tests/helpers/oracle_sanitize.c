/* Drives every entry point of the CPU oracle on small inputs of every model
 * kind and precision, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only): any out-of-bounds access,
 * leak, overflow or other undefined behaviour aborts the run. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/cmo.h"

static int run(cmo_model *m, cmo_sweep *s) {
  const int64_t S = s->n_settings;
  const uint64_t runs = (uint64_t)S * s->trials;
  const int width = cmo_state_width(m);
  cmo_result r = {0};
  r.hist = calloc((size_t)S * 2 * s->n_bins, sizeof(uint64_t));
  r.stats = calloc((size_t)S * CMO_NSTAT, sizeof(uint64_t));
  r.score = calloc((size_t)S, sizeof(double));
  r.best = calloc(2, sizeof(int64_t));
  r.run_choice = calloc(runs, 1);
  r.run_step = calloc(runs, sizeof(uint32_t));
  r.run_flag = calloc(runs, 1);
  r.run_state = calloc(runs * (size_t)width, sizeof(double));
  int rc = cmo_run(m, s, &r, 2);
  double *traj = calloc((size_t)s->max_steps * width, sizeof(double));
  int8_t ch;
  uint8_t fl;
  if (!rc && cmo_trajectory(m, s, S - 1, s->trials - 1, traj, &ch, &fl) == 0) rc = 1;
  if (!rc && (m->kind == CMO_DDM || m->kind == CMO_LCA)) {
    const uint32_t every = s->max_steps > 3 ? 3 : 1;
    int64_t *tc = calloc((size_t)S * (s->max_steps / every) * CMO_TC_WORDS, sizeof(int64_t));
    rc = cmo_timecourse(m, s, every, tc, 2);
    free(tc);
  }
  free(traj);
  free(r.hist); free(r.stats); free(r.score); free(r.best);
  free(r.run_choice); free(r.run_step); free(r.run_flag); free(r.run_state);
  return rc;
}

int main(void) {
  int fails = 0;
  double lca_w[40], grid2[6] = {0.0, 1.0, 2.5, 1.0, 5.0, 0.3};
  for (int i = 0; i < 40; ++i) lca_w[i] = 2.0 * sin(1.7 * i + 0.3);
  enum { NU = 64 };
  static double rnn_w[NU * NU + 2 * NU];
  for (int i = 0; i < NU * NU + 2 * NU; ++i) rnn_w[i] = 0.25 * sin(0.37 * i + 1.1);
  for (int prec = 0; prec < 2; ++prec) {
    double pd[CMO_DDM_NPARAM] = {0.01, 0.3, 1.0, 1.0, 0.0, 0.2};
    double drifts[3] = {-0.2, 0.1, 0.5};
    cmo_model m = {CMO_DDM, prec, 1, 1, 1, pd, CMO_DDM_NPARAM, NULL, 0};
    cmo_sweep s = {drifts, 3, 37, 5, 301, 7, 0.0, 0.0, 1e-10};
    fails += run(&m, &s) != 0;
    double pl[CMO_LCA_NPARAM] = {0.1, 0.5, 1.0, 0.1, 0.8, 0.0, 1.0, -4.0, 0.0, 0.0};
    cmo_model ml = {CMO_LCA, prec, 2, 9, 2, pl, CMO_LCA_NPARAM, lca_w, 40};
    cmo_sweep sl = {grid2, 3, 23, 7, 200, 20, 1.0, 0.1, 1e-10};
    fails += run(&ml, &sl) != 0;
    pl[CMO_LCA_NONNEG] = 1.0;
    fails += run(&ml, &sl) != 0;
    double pp[CMO_LOOP_NPARAM] = {0.1, 0.5, 1.0, 0.1, 0.8, 0.0, 1.0, -4.0, 0.0, 0.0, 3, 5.0, 2, 0.01};
    cmo_model mp = {CMO_LOOP, prec, 2, 9, 0, pp, CMO_LOOP_NPARAM, lca_w, 40};
    cmo_sweep sp = {NULL, 1, 11, 9, 60, 6, 0.0, 0.0, 1e-10};
    fails += run(&mp, &sp) != 0;
  }
  for (int prec = 0; prec < 3; prec += 2) {
    double pr[CMO_RNN_NPARAM] = {0.05, 0.05, 1.0, 1.0, 0.0};
    double gains[2] = {0.5, 1.5};
    cmo_model m = {CMO_RNN, prec, NU, 1, 1, pr, CMO_RNN_NPARAM, rnn_w, NU * NU + 2 * NU};
    cmo_sweep s = {gains, 2, 5, 3, 40, 8, 0.0, 0.0, 1e-10};
    fails += run(&m, &s) != 0;
  }
  double lo[400], up[400];
  fails += cmo_ddm_density(0.003, 0.1, 1.0, 0.1, 57, 400, 1e-15, lo, up) != 0;
  printf("oracle sanitizer driver: %d failures\n", fails);
  return fails != 0;
}
