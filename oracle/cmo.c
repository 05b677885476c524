/*
 * cmo.c -- plain FP64 CPU oracle for batched cognitive-model simulation.
 *
 * TEST INFRASTRUCTURE ONLY: called by tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the HIP library.
 *
 * What it computes (the Distill paper, arXiv 2110.15425):
 *  - the scheduling loop of Sec. 2.2: trials run one after another, trial t
 *    reads input number t mod len(inputs), and a trial iterates the model's
 *    mechanisms until its end condition holds (here: a threshold crossing or
 *    the step cap);
 *  - the grid evaluation of Sec. 3.6: every (setting, trial) pair is an
 *    independent evaluation with its own random stream, so parallel workers
 *    draw identical numbers (the PRNG-per-evaluation requirement of Sec. 3.6);
 *  - the mechanisms named in Sec. 4.4: the drift-diffusion model (DDM) and
 *    the leaky competing accumulator (LCA) whose update with leak 0 and
 *    offset 0 coincides with the DDM's; the logistic transfer and
 *    weight-matrix projections of Sec. 3.4.2;
 *  - outcome histograms and the best control allocation of Sec. 2.1, with
 *    random tie-breaking among equal-cost choices (Sec. 3.3).
 * The paper prints no equations for the mechanisms; the readings used here
 * (Euler-Maruyama noise scaling, >= at threshold, integer-step decision
 * times, linear LCA, the conflict network's logistic drive, the rate
 * network's centred readout, Philox streams, Box-Muller normals) are stated
 * where they are used, and the tests pin each part of this file to values
 * fixed by the mathematics (closed forms, special cases, brute force).
 *
 * Everything is evaluated in the order written, in FP64 unless a precision
 * mode says otherwise, built with -ffp-contract=off so no FMA is formed.
 * Parallelism: runs are simulated independently (OpenMP); the reduction into
 * histograms and statistics is a separate serial integer pass.
 */
#include "cmo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies, with    */
/* the key bumped by the Weyl constants between rounds.                      */
/* ------------------------------------------------------------------------ */
void cmo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* one block of the stream keyed by the seed, counter (k, trial, setting, stream) */
static void block(uint64_t seed, uint32_t k, uint64_t trial, uint64_t setting,
                  uint32_t stream, uint32_t w[4]) {
  uint32_t ctr[4] = {k, (uint32_t)trial, (uint32_t)setting, stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  cmo_philox4x32_10(ctr, key, w);
}

/* Two standard normals from one block: 53-bit uniforms in (0,1], Box-Muller. */
void cmo_normals64(const uint32_t w[4], double z[2]) {
  uint64_t ma = ((((uint64_t)w[1]) << 32) | (uint64_t)w[0]) >> 11;
  uint64_t mb = ((((uint64_t)w[3]) << 32) | (uint64_t)w[2]) >> 11;
  double ua = (double)(ma + 1u) * 0x1p-53;
  double ub = (double)(mb + 1u) * 0x1p-53;
  double rho = sqrt(-2.0 * log(ua));
  double phi = 6.283185307179586 * ub;
  z[0] = rho * cos(phi);
  z[1] = rho * sin(phi);
}

/* FP32 variant: the top 24 bits of the same words. */
void cmo_normals32(const uint32_t w[4], float z[2]) {
  float ua = (float)((w[1] >> 8) + 1u) * 0x1p-24f;
  float ub = (float)((w[3] >> 8) + 1u) * 0x1p-24f;
  float rho = sqrtf(-2.0f * logf(ua));
  float phi = 6.28318548f * ub;
  z[0] = rho * cosf(phi);
  z[1] = rho * sinf(phi);
}

uint16_t cmo_bf16_bits(double v) {
  float f = (float)v;
  uint32_t bits;
  memcpy(&bits, &f, sizeof bits);
  if ((bits & 0x7F800000u) == 0x7F800000u && (bits & 0x007FFFFFu))
    return (uint16_t)((bits >> 16) | 0x0040u); /* quiet NaN */
  uint32_t lsb = (bits >> 16) & 1u;
  bits += 0x7FFFu + lsb;
  return (uint16_t)(bits >> 16);
}

static float bf16_value(float f) {
  uint16_t h = cmo_bf16_bits((double)f);
  uint32_t bits = ((uint32_t)h) << 16;
  float r;
  memcpy(&r, &bits, sizeof r);
  return r;
}

static double logistic(double v) { return 1.0 / (1.0 + exp(-v)); }

/* ------------------------------------------------------------------------ */
/* Mechanism updates (Euler-Maruyama).                                       */
/* ------------------------------------------------------------------------ */
double cmo_ddm_update(double x, double a, double b, double z) { return (x + a) + b * z; }

void cmo_lca_update(const double x[2], const double in[2], double leak, double comp,
                    double dt, double b, const double z[2], double out[2]) {
  /* simultaneous update: both units read the previous state */
  out[0] = (x[0] + (((in[0] - leak * x[0]) - comp * x[1]) * dt)) + b * z[0];
  out[1] = (x[1] + (((in[1] - leak * x[1]) - comp * x[0]) * dt)) + b * z[1];
}

/* Conflict network: two one-hot 3-unit inputs, two 4-unit logistic hidden
 * layers whose gain is multiplied by the pathway's control signal, and
 * [2x4] projections from each hidden layer onto the 2 accumulators. */
void cmo_conflict_drive(const double *wt, double gain, double bias, double offset,
                        double cA, double cB, double drive[9][2]) {
  const double *WA = wt, *WB = wt + 12, *OA = wt + 24, *OB = wt + 32;
  for (int stim = 0; stim < 9; ++stim) {
    int a = stim / 3, b = stim % 3;
    double hA[4], hB[4];
    for (int k = 0; k < 4; ++k) {
      hA[k] = logistic((cA * gain) * (WA[k * 3 + a] + bias));
      hB[k] = logistic((cB * gain) * (WB[k * 3 + b] + bias));
    }
    for (int j = 0; j < 2; ++j) {
      double sA = 0.0, sB = 0.0;
      for (int k = 0; k < 4; ++k) sA = sA + OA[j * 4 + k] * hA[k];
      for (int k = 0; k < 4; ++k) sB = sB + OB[j * 4 + k] * hB[k];
      drive[stim][j] = (sA + sB) + offset;
    }
  }
}

void cmo_conflict_correct(const double *wt, double gain, double bias, int32_t correct[9]) {
  const double *WA = wt, *OA = wt + 24;
  for (int stim = 0; stim < 9; ++stim) {
    int a = stim / 3;
    double s[2];
    for (int j = 0; j < 2; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 4; ++k) acc = acc + OA[j * 4 + k] * logistic(gain * (WA[k * 3 + a] + bias));
      s[j] = acc;
    }
    correct[stim] = (s[1] > s[0]) ? 1 : 0;
  }
}

int cmo_state_width(const cmo_model *m) {
  if (m->kind == CMO_DDM) return 1;
  if (m->kind == CMO_LCA || m->kind == CMO_LOOP) return 2;
  return 2 + m->n_units;
}

/* ------------------------------------------------------------------------ */
/* One run.                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  int8_t choice;
  uint32_t steps;
  uint8_t flag;
} run_out;

static double param(const cmo_model *m, int i) { return m->params[i]; }

static double signal(const cmo_model *m, const cmo_sweep *s, int64_t setting, int i,
                     double dflt) {
  if (m->n_signals <= i) return dflt;
  return s->grid[setting * m->n_signals + i];
}

static int near(double q, double th, double eps) { return fabs(q - th) < eps; }

static run_out run_ddm(const cmo_model *m, const cmo_sweep *s, int64_t setting,
                       uint64_t trial, double *state, double *traj) {
  double dt = param(m, CMO_DDM_DT);
  double drift = signal(m, s, setting, 0, param(m, CMO_DDM_DRIFT));
  double noise = param(m, CMO_DDM_NOISE), th = param(m, CMO_DDM_THRESH);
  double a = drift * dt, b = noise * sqrt(dt);
  float af = (float)a, bf = (float)b;
  double x = param(m, CMO_DDM_START), eps = s->flag_eps;
  run_out o = {-1, s->max_steps, 0};
  double z64[2] = {0, 0};
  float z32[2] = {0, 0};
  for (uint32_t n = 1; n <= s->max_steps; ++n) {
    uint32_t e = (n - 1) & 1u;
    if (e == 0) {
      uint32_t w[4];
      block(s->seed, (n - 1) >> 1, trial, (uint64_t)setting, 0, w);
      if (m->precision == CMO_FP64) cmo_normals64(w, z64);
      else cmo_normals32(w, z32);
    }
    if (m->precision == CMO_FP64) {
      x = cmo_ddm_update(x, a, b, z64[e]);
    } else {
      float inc = af + bf * z32[e];
      x = x + (double)inc;
    }
    if (traj) traj[n - 1] = x;
    if (near(x, th, eps) || near(x, -th, eps)) o.flag = 1;
    if (x >= th) { o.choice = 1; o.steps = n; break; }
    if (x <= -th) { o.choice = 0; o.steps = n; break; }
  }
  if (state) state[0] = x;
  return o;
}

static run_out run_lca(const cmo_model *m, const cmo_sweep *s, int64_t setting,
                       uint64_t trial, double *state, double *traj) {
  double dt = param(m, CMO_LCA_DT), leak = param(m, CMO_LCA_LEAK);
  double comp = param(m, CMO_LCA_COMP), noise = param(m, CMO_LCA_NOISE);
  double th = param(m, CMO_LCA_THRESH), eps = s->flag_eps;
  int nonneg = param(m, CMO_LCA_NONNEG) != 0.0;
  double cA = signal(m, s, setting, 0, 1.0), cB = signal(m, s, setting, 1, 1.0);
  double drive[9][2];
  /* loop-invariant feed-forward part, evaluated once per setting */
  cmo_conflict_drive(m->weights, param(m, CMO_LCA_HID_GAIN), param(m, CMO_LCA_HID_BIAS),
                     param(m, CMO_LCA_OFFSET), cA, cB, drive);
  int stim = (int)(trial % (uint64_t)m->n_stimuli);
  double in[2] = {drive[stim][0], drive[stim][1]};
  double b = noise * sqrt(dt);
  float inf[2] = {(float)in[0], (float)in[1]};
  float leakf = (float)leak, compf = (float)comp, dtf = (float)dt, bf = (float)b;
  double x[2] = {0.0, 0.0};
  run_out o = {-1, s->max_steps, 0};
  for (uint32_t n = 1; n <= s->max_steps; ++n) {
    uint32_t w[4];
    block(s->seed, n - 1, trial, (uint64_t)setting, 0, w);
    double y[2];
    if (m->precision == CMO_FP64) {
      double z[2];
      cmo_normals64(w, z);
      cmo_lca_update(x, in, leak, comp, dt, b, z, y);
    } else {
      float z[2];
      cmo_normals32(w, z);
      float xf0 = (float)x[0], xf1 = (float)x[1];
      float inc0 = (((inf[0] - leakf * xf0) - compf * xf1) * dtf) + bf * z[0];
      float inc1 = (((inf[1] - leakf * xf1) - compf * xf0) * dtf) + bf * z[1];
      y[0] = x[0] + (double)inc0;
      y[1] = x[1] + (double)inc1;
    }
    if (nonneg) {
      if (y[0] < 0.0) y[0] = 0.0;
      if (y[1] < 0.0) y[1] = 0.0;
    }
    x[0] = y[0];
    x[1] = y[1];
    if (traj) { traj[2 * (n - 1)] = x[0]; traj[2 * (n - 1) + 1] = x[1]; }
    if (near(x[0], th, eps) || near(x[1], th, eps)) o.flag = 1;
    double mx = x[0] > x[1] ? x[0] : x[1];
    if (mx >= th) {
      o.choice = (x[1] > x[0]) ? 1 : 0;
      if (fabs(x[0] - x[1]) < eps) o.flag = 1;
      o.steps = n;
      break;
    }
  }
  if (state) { state[0] = x[0]; state[1] = x[1]; }
  return o;
}

/* Transposed weight copies, built once per sweep, so that p_i accumulates
 * over j in ascending order while the inner loop runs over i (the same sums
 * in the same order, only vectorisable). */
typedef struct {
  double *WT;  /* FP64 mode */
  float *WTf;  /* FP32 / BF16 modes: float(W), bf16-rounded in BF16 mode */
  double *loop_drive; /* closed loop: drive [allocation][stimulus][2] */
  int32_t correct[9];
} rnn_ctx;

static double loop_level(double amax, uint32_t L, uint32_t i) {
  return L == 1 ? amax : (amax * (double)i) / (double)(L - 1);
}

static void rnn_ctx_init(const cmo_model *m, rnn_ctx *c) {
  const int nu = m->n_units;
  const double *W = m->weights;
  c->WT = NULL;
  c->WTf = NULL;
  c->loop_drive = NULL;
  if (m->kind == CMO_LOOP) {
    /* the drive of every allocation, evaluated once per sweep (loop-invariant) */
    const uint32_t L = (uint32_t)m->params[CMO_LOOP_LEVELS], J = L * L;
    const double amax = m->params[CMO_LOOP_AMAX];
    c->loop_drive = malloc(sizeof(double) * (size_t)J * 18);
    for (uint32_t j = 0; j < J; ++j)
      cmo_conflict_drive(m->weights, m->params[CMO_LCA_HID_GAIN], m->params[CMO_LCA_HID_BIAS],
                         m->params[CMO_LCA_OFFSET], loop_level(amax, L, j / L),
                         loop_level(amax, L, j % L), (double(*)[2])(c->loop_drive + 18 * (size_t)j));
    cmo_conflict_correct(m->weights, m->params[CMO_LCA_HID_GAIN], m->params[CMO_LCA_HID_BIAS],
                         c->correct);
    return;
  }
  if (m->kind != CMO_RNN) return;
  if (m->precision == CMO_FP64) {
    c->WT = malloc(sizeof(double) * (size_t)nu * nu);
    for (int i = 0; i < nu; ++i)
      for (int j = 0; j < nu; ++j) c->WT[(size_t)j * nu + i] = W[(size_t)i * nu + j];
  } else {
    c->WTf = malloc(sizeof(float) * (size_t)nu * nu);
    for (int i = 0; i < nu; ++i)
      for (int j = 0; j < nu; ++j) {
        float wf = (float)W[(size_t)i * nu + j];
        c->WTf[(size_t)j * nu + i] = (m->precision == CMO_BF16_PROJ) ? bf16_value(wf) : wf;
      }
  }
}

static void rnn_ctx_free(rnn_ctx *c) {
  free(c->WT);
  free(c->WTf);
  free(c->loop_drive);
}

static run_out run_rnn(const cmo_model *m, const cmo_sweep *s, const rnn_ctx *ctx,
                       int64_t setting, uint64_t trial, double *state, double *traj) {
  const int nu = m->n_units;
  const double *R = m->weights + (int64_t)nu * nu;
  const double *WT = ctx->WT;
  const float *WTf = ctx->WTf;
  double dt = param(m, CMO_RNN_DT), noise = param(m, CMO_RNN_NOISE);
  double th = param(m, CMO_RNN_THRESH), eps = s->flag_eps;
  double g = signal(m, s, setting, 0, param(m, CMO_RNN_INPUT_GAIN));
  double b = noise * sqrt(dt);
  float dtf = (float)dt, gf = (float)g, bf = (float)b;
  const int prec = m->precision;
  double *x = calloc((size_t)nu, sizeof(double));
  double *r = malloc(sizeof(double) * (size_t)nu);
  double *p = malloc(sizeof(double) * (size_t)nu);
  double *u = malloc(sizeof(double) * (size_t)nu);
  double *xi = malloc(sizeof(double) * (size_t)nu);
  float *rf = malloc(sizeof(float) * (size_t)nu);
  float *rq = malloc(sizeof(float) * (size_t)nu);
  float *pf = malloc(sizeof(float) * (size_t)nu);
  float *uf = malloc(sizeof(float) * (size_t)nu);
  float *xif = malloc(sizeof(float) * (size_t)nu);
  /* per-run input drive, N(0,1) per unit */
  for (int mm = 0; mm < nu / 2; ++mm) {
    uint32_t w[4];
    block(s->seed, (uint32_t)mm, trial, (uint64_t)setting, CMO_STREAM_DRIVE, w);
    if (prec == CMO_FP64) {
      double z[2];
      cmo_normals64(w, z);
      u[2 * mm] = z[0];
      u[2 * mm + 1] = z[1];
    } else {
      float z[2];
      cmo_normals32(w, z);
      uf[2 * mm] = z[0];
      uf[2 * mm + 1] = z[1];
    }
  }
  double y[2] = {0.0, 0.0};
  run_out o = {-1, s->max_steps, 0};
  for (uint32_t n = 1; n <= s->max_steps; ++n) {
    /* noise for this step: unit pair (2m, 2m+1) reads stream m */
    for (int mm = 0; mm < nu / 2; ++mm) {
      uint32_t w[4];
      block(s->seed, n - 1, trial, (uint64_t)setting, (uint32_t)mm, w);
      if (prec == CMO_FP64) {
        double z[2];
        cmo_normals64(w, z);
        xi[2 * mm] = z[0];
        xi[2 * mm + 1] = z[1];
      } else {
        float z[2];
        cmo_normals32(w, z);
        xif[2 * mm] = z[0];
        xif[2 * mm + 1] = z[1];
      }
    }
    if (prec == CMO_FP64) {
      for (int j = 0; j < nu; ++j) r[j] = logistic(x[j]);
      for (int i = 0; i < nu; ++i) p[i] = 0.0;
      for (int j = 0; j < nu; ++j) {
        const double rj = r[j], *col = WT + (size_t)j * nu;
        for (int i = 0; i < nu; ++i) p[i] = p[i] + col[i] * rj;
      }
      double acc[2];
      for (int c = 0; c < 2; ++c) {
        double a = 0.0;
        for (int j = 0; j < nu; ++j) a = a + R[(size_t)c * nu + j] * (r[j] - 0.5);
        acc[c] = a;
      }
      for (int i = 0; i < nu; ++i) x[i] = (x[i] + dt * ((p[i] - x[i]) + g * u[i])) + b * xi[i];
      y[0] = y[0] + dt * acc[0];
      y[1] = y[1] + dt * acc[1];
    } else {
      for (int j = 0; j < nu; ++j) {
        float xf = (float)x[j];
        rf[j] = 1.0f / (1.0f + expf(-xf));
        rq[j] = (prec == CMO_BF16_PROJ) ? bf16_value(rf[j]) : rf[j];
      }
      for (int i = 0; i < nu; ++i) pf[i] = 0.0f;
      for (int j = 0; j < nu; ++j) {
        const float rj = rq[j], *col = WTf + (size_t)j * nu;
        for (int i = 0; i < nu; ++i) pf[i] = pf[i] + col[i] * rj;
      }
      float acc[2];
      for (int c = 0; c < 2; ++c) {
        float a = 0.0f;
        for (int j = 0; j < nu; ++j) a = a + (float)R[(size_t)c * nu + j] * (rf[j] - 0.5f);
        acc[c] = a;
      }
      for (int i = 0; i < nu; ++i) {
        float xf = (float)x[i];
        float inc = dtf * ((pf[i] - xf) + gf * uf[i]) + bf * xif[i];
        x[i] = x[i] + (double)inc;
      }
      y[0] = y[0] + (double)(dtf * acc[0]);
      y[1] = y[1] + (double)(dtf * acc[1]);
    }
    if (traj) {
      double *row = traj + (size_t)(n - 1) * (2 + nu);
      row[0] = y[0];
      row[1] = y[1];
      for (int i = 0; i < nu; ++i) row[2 + i] = x[i];
    }
    if (near(y[0], th, eps) || near(y[1], th, eps)) o.flag = 1;
    double mx = y[0] > y[1] ? y[0] : y[1];
    if (mx >= th) {
      o.choice = (y[1] > y[0]) ? 1 : 0;
      if (fabs(y[0] - y[1]) < eps) o.flag = 1;
      o.steps = n;
      break;
    }
  }
  if (state) {
    state[0] = y[0];
    state[1] = y[1];
    for (int i = 0; i < nu; ++i) state[2 + i] = x[i];
  }
  free(x); free(r); free(p); free(u); free(xi);
  free(rf); free(rq); free(pf); free(uf); free(xif);
  return o;
}

/* One LCA step from state x with drive in and the normals of block w, in the
 * model's precision (the same arithmetic as run_lca), NONNEG clipping
 * included. */
static void loop_step(const cmo_model *m, const double x[2], const double in[2], const uint32_t w[4],
                      double y[2]) {
  double dt = param(m, CMO_LCA_DT), leak = param(m, CMO_LCA_LEAK);
  double comp = param(m, CMO_LCA_COMP), b = param(m, CMO_LCA_NOISE) * sqrt(dt);
  if (m->precision == CMO_FP64) {
    double z[2];
    cmo_normals64(w, z);
    cmo_lca_update(x, in, leak, comp, dt, b, z, y);
  } else {
    float z[2];
    cmo_normals32(w, z);
    float inf0 = (float)in[0], inf1 = (float)in[1];
    float leakf = (float)leak, compf = (float)comp, dtf = (float)dt, bf = (float)b;
    float xf0 = (float)x[0], xf1 = (float)x[1];
    float inc0 = (((inf0 - leakf * xf0) - compf * xf1) * dtf) + bf * z[0];
    float inc1 = (((inf1 - leakf * xf1) - compf * xf0) * dtf) + bf * z[1];
    y[0] = x[0] + (double)inc0;
    y[1] = x[1] + (double)inc1;
  }
  if (param(m, CMO_LCA_NONNEG) != 0.0) {
    if (y[0] < 0.0) y[0] = 0.0;
    if (y[1] < 0.0) y[1] = 0.0;
  }
}

/* Closed-loop control of the conflict network: before every step the control
 * node evaluates each allocation (c_A, c_B) of the L x L level grid by M
 * sampled one-step look-aheads of the accumulators (each with its own random
 * stream), scores it as cost * (c_A^2 + c_B^2) minus the mean gain in
 * evidence for the correct response, x_c - x_w, and picks the lowest score
 * (ties: a random pick, the smallest Philox priority); the step itself then
 * runs with the chosen allocation on the run's own stream.  State carries
 * across steps, and the search is nested inside each step, as in the
 * predator-prey control loop (Sec. 2.1); evaluations of the allocations and
 * samples are independent (Sec. 3.6).  A run is flagged when the best and
 * second-best scores differ by less than flag_eps without being equal. */
static run_out run_loop(const cmo_model *m, const cmo_sweep *s, const rnn_ctx *ctx,
                        int64_t setting, uint64_t trial, double *state, double *traj) {
  const double th = param(m, CMO_LCA_THRESH), eps = s->flag_eps;
  const uint32_t L = (uint32_t)param(m, CMO_LOOP_LEVELS), J = L * L;
  const uint32_t M = (uint32_t)param(m, CMO_LOOP_SAMPLES);
  const double amax = param(m, CMO_LOOP_AMAX);
  const double kappa = signal(m, s, setting, 0, param(m, CMO_LOOP_COST));
  const int stim = (int)(trial % 9u);
  const int c = ctx->correct[stim], o = 1 - c;
  const uint32_t key[2] = {(uint32_t)s->seed, (uint32_t)(s->seed >> 32)};
  double x[2] = {0.0, 0.0};
  run_out out = {-1, s->max_steps, 0};
  for (uint32_t n = 1; n <= s->max_steps; ++n) {
    double bestV = INFINITY, secondV = INFINITY;
    uint32_t best = 0, best_prio = 0;
    for (uint32_t j = 0; j < J; ++j) {
      const double *in = ctx->loop_drive + (18 * (size_t)j + 2 * (size_t)stim);
      double gsum = 0.0;
      for (uint32_t mm = 0; mm < M; ++mm) {
        uint32_t w[4];
        block(s->seed, n - 1, trial, (uint64_t)setting, CMO_STREAM_LOOK | (j * M + mm), w);
        double y[2];
        loop_step(m, x, in, w, y);
        gsum = gsum + ((y[c] - y[o]) - (x[c] - x[o]));
      }
      const double cA = loop_level(amax, L, j / L), cB = loop_level(amax, L, j % L);
      const double V = kappa * (cA * cA + cB * cB) - gsum / (double)M;
      uint32_t ctr[4] = {n - 1, (uint32_t)trial, (uint32_t)setting, CMO_STREAM_PICK | j}, pw[4];
      if (V < bestV) {
        secondV = bestV;
        bestV = V;
        best = j;
        cmo_philox4x32_10(ctr, key, pw);
        best_prio = pw[0];
      } else if (V == bestV) {
        secondV = V;
        cmo_philox4x32_10(ctr, key, pw);
        if (pw[0] < best_prio) { /* allocations visited ascending: equal priority keeps the smaller */
          best = j;
          best_prio = pw[0];
        }
      } else if (V < secondV) {
        secondV = V;
      }
    }
    if (secondV > bestV && secondV - bestV < eps) out.flag = 1;
    uint32_t w[4];
    block(s->seed, n - 1, trial, (uint64_t)setting, 0, w);
    double y[2];
    loop_step(m, x, ctx->loop_drive + (18 * (size_t)best + 2 * (size_t)stim), w, y);
    x[0] = y[0];
    x[1] = y[1];
    if (traj) { traj[2 * (n - 1)] = x[0]; traj[2 * (n - 1) + 1] = x[1]; }
    if (near(x[0], th, eps) || near(x[1], th, eps)) out.flag = 1;
    double mx = x[0] > x[1] ? x[0] : x[1];
    if (mx >= th) {
      out.choice = (x[1] > x[0]) ? 1 : 0;
      if (fabs(x[0] - x[1]) < eps) out.flag = 1;
      out.steps = n;
      break;
    }
  }
  if (state) { state[0] = x[0]; state[1] = x[1]; }
  return out;
}

static run_out run_one(const cmo_model *m, const cmo_sweep *s, const rnn_ctx *ctx,
                       int64_t setting, uint64_t trial, double *state, double *traj) {
  if (m->kind == CMO_DDM) return run_ddm(m, s, setting, trial, state, traj);
  if (m->kind == CMO_LCA) return run_lca(m, s, setting, trial, state, traj);
  if (m->kind == CMO_LOOP) return run_loop(m, s, ctx, setting, trial, state, traj);
  return run_rnn(m, s, ctx, setting, trial, state, traj);
}

/* ------------------------------------------------------------------------ */
/* Validation                                                                */
/* ------------------------------------------------------------------------ */
static int invalid(const cmo_model *m, const cmo_sweep *s) {
  if (!m || !s || !m->params) return 1;
  if (s->n_settings < 1 || s->trials < 1 || s->trials > 0xFFFFFFFFull) return 1;
  if ((uint64_t)s->n_settings > 0xFFFFFFFEull) return 1;
  if (s->max_steps < 1 || s->n_bins < 1 || s->n_bins > s->max_steps) return 1;
  if (m->n_signals > 0 && !s->grid) return 1;
  if (m->kind == CMO_DDM) {
    if (m->n_params < CMO_DDM_NPARAM || m->n_stimuli != 1 || m->n_signals > 1) return 1;
    if (m->precision == CMO_BF16_PROJ) return 1;
    const double *p = m->params;
    if (!(p[CMO_DDM_DT] > 0) || !(p[CMO_DDM_NOISE] >= 0) || !(p[CMO_DDM_THRESH] > 0)) return 1;
    if (!(fabs(p[CMO_DDM_START]) < p[CMO_DDM_THRESH])) return 1;
  } else if (m->kind == CMO_LCA) {
    if (m->n_params < CMO_LCA_NPARAM || m->n_stimuli != 9 || m->n_units != 2) return 1;
    if (m->n_signals != 0 && m->n_signals != 2) return 1;
    if (!m->weights || m->n_weights < 40 || m->precision == CMO_BF16_PROJ) return 1;
    const double *p = m->params;
    if (!(p[CMO_LCA_DT] > 0) || !(p[CMO_LCA_NOISE] >= 0) || !(p[CMO_LCA_THRESH] > 0)) return 1;
  } else if (m->kind == CMO_LOOP) {
    if (m->n_params < CMO_LOOP_NPARAM || m->n_stimuli != 9 || m->n_units != 2) return 1;
    if (m->n_signals > 1 || !m->weights || m->n_weights < 40) return 1;
    if (m->precision == CMO_BF16_PROJ) return 1;
    const double *p = m->params;
    if (!(p[CMO_LCA_DT] > 0) || !(p[CMO_LCA_NOISE] >= 0) || !(p[CMO_LCA_THRESH] > 0)) return 1;
    const double L = p[CMO_LOOP_LEVELS], M = p[CMO_LOOP_SAMPLES];
    if (!(L >= 1 && L <= 4096 && L == floor(L)) || !(M >= 1 && M <= 4096 && M == floor(M))) return 1;
    if (L * L * M >= 1073741824.0 || !(p[CMO_LOOP_AMAX] >= 0)) return 1;
  } else if (m->kind == CMO_RNN) {
    if (m->n_params < CMO_RNN_NPARAM || m->n_stimuli != 1 || m->n_signals > 1) return 1;
    if (m->n_units < 2 || m->n_units > 1024 || (m->n_units & 1)) return 1;
    if (!m->weights || m->n_weights < (int64_t)m->n_units * m->n_units + 2 * m->n_units) return 1;
    const double *p = m->params;
    if (!(p[CMO_RNN_DT] > 0) || !(p[CMO_RNN_NOISE] >= 0) || !(p[CMO_RNN_THRESH] > 0)) return 1;
  } else {
    return 1;
  }
  return 0;
}

/* "correct" response per stimulus: DDM upper boundary; conflict network the
 * noise-free response of the relevant pathway; the rate network has none. */
static void correct_table(const cmo_model *m, int32_t correct[9]) {
  for (int i = 0; i < 9; ++i) correct[i] = -1;
  if (m->kind == CMO_DDM) correct[0] = 1;
  else if (m->kind == CMO_LCA || m->kind == CMO_LOOP)
    cmo_conflict_correct(m->weights, m->params[CMO_LCA_HID_GAIN], m->params[CMO_LCA_HID_BIAS],
                         correct);
}

uint32_t cmo_trajectory(const cmo_model *m, const cmo_sweep *s, int64_t setting, uint64_t trial,
                        double *states, int8_t *choice, uint8_t *flag) {
  if (invalid(m, s) || setting < 0 || setting >= s->n_settings || trial >= s->trials) return 0;
  rnn_ctx ctx;
  rnn_ctx_init(m, &ctx);
  run_out o = run_one(m, s, &ctx, setting, trial, NULL, states);
  rnn_ctx_free(&ctx);
  if (choice) *choice = o.choice;
  if (flag) *flag = o.flag;
  return o.steps;
}

/* ------------------------------------------------------------------------ */
/* Time course: ensemble statistics of the state at sample steps, the         */
/* dynamics over time that modellers study beside final outcomes (Sec. 1,     */
/* Sec. 2.1), including the conflict energy of the two mutually inhibiting    */
/* response units (the Stroop model's decision energy, Sec. 4.4).  Sums are   */
/* integers of fixed-point values, so they do not depend on summation order.  */
/* ------------------------------------------------------------------------ */
int64_t cmo_tc_quant(double v) {
  const double lim = 4611686018427387904.0; /* 2^62 */
  double t = nearbyint(ldexp(v, 32));
  if (t > lim) t = lim;
  if (t < -lim) t = -lim;
  return (int64_t)t;
}

static void tc_add(int64_t *w, double x0, double x1, double comp) {
  uint64_t *u = (uint64_t *)w; /* wrap-around sums */
  u[0] += 1u;
  u[1] += (uint64_t)cmo_tc_quant(x0);
  u[2] += (uint64_t)cmo_tc_quant(x1);
  u[3] += (uint64_t)cmo_tc_quant(x0 * x0);
  u[4] += (uint64_t)cmo_tc_quant(x1 * x1);
  u[5] += (uint64_t)cmo_tc_quant(comp * (x0 * x1));
}

int cmo_timecourse(const cmo_model *m, const cmo_sweep *s, uint32_t every, int64_t *tc,
                   int n_threads) {
  if (invalid(m, s) || !tc || every < 1 || every > s->max_steps) return 1;
  if (m->kind != CMO_DDM && m->kind != CMO_LCA) return 1;
  const int64_t S = s->n_settings;
  const uint64_t T = s->trials;
  const uint32_t K = s->max_steps / every, N = s->max_steps;
  const int width = cmo_state_width(m);
  const double comp = m->kind == CMO_LCA ? param(m, CMO_LCA_COMP) : 0.0;
  memset(tc, 0, sizeof(int64_t) * (size_t)S * K * CMO_TC_WORDS);
  int fail = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t setting = 0; setting < S; ++setting) {
    double *traj = malloc(sizeof(double) * (size_t)N * width);
    if (!traj) {
      fail = 1;
      continue;
    }
    int64_t *row = tc + (size_t)setting * K * CMO_TC_WORDS;
    for (uint64_t trial = 0; trial < T; ++trial) {
      run_out o = run_one(m, s, NULL, setting, trial, NULL, traj);
      for (uint32_t k = 1; k <= K && (uint64_t)k * every <= o.steps; ++k) {
        const double *x = traj + (size_t)(k * every - 1) * width;
        tc_add(row + (size_t)(k - 1) * CMO_TC_WORDS, x[0], width > 1 ? x[1] : 0.0, comp);
      }
    }
    free(traj);
  }
  return fail ? 2 : 0;
}

/* ------------------------------------------------------------------------ */
/* First-passage distribution of the discretised DDM by propagating the      */
/* survivor mass on M cells of (-theta, theta): the walk's transition from   */
/* a point is Gaussian, so the mass a cell receives is a difference of       */
/* normal CDFs at its edges and the mass absorbed is a normal tail.  The     */
/* first step leaves the exact start point, later steps the cell centres.    */
/* ------------------------------------------------------------------------ */
static double Phi(double x) { return 0.5 * erfc(-x * 0.70710678118654752440); }

int cmo_ddm_density(double a, double b, double theta, double start, int cells, int max_steps,
                    double tol, double *lower, double *upper) {
  if (cells < 2 || max_steps < 1 || !(b > 0) || !(theta > 0) || !(fabs(start) < theta)) return 1;
  const int M = cells;
  const double h = (2.0 * theta) / (double)M;
  double *f = malloc(sizeof(double) * (size_t)(2 * M - 1));
  double *up = malloc(sizeof(double) * (size_t)M);
  double *lo = malloc(sizeof(double) * (size_t)M);
  double *mass = malloc(sizeof(double) * (size_t)M);
  double *next = malloc(sizeof(double) * (size_t)M);
  if (!f || !up || !lo || !mass || !next) return 2;
  for (int d = 0; d < 2 * M - 1; ++d) {
    double k = (double)(d - (M - 1));
    f[d] = Phi(((k + 0.5) * h - a) / b) - Phi(((k - 0.5) * h - a) / b);
  }
  for (int i = 0; i < M; ++i) {
    double c = -theta + ((double)i + 0.5) * h;
    up[i] = Phi(-((theta - c) - a) / b);
    lo[i] = Phi(((-theta - c) - a) / b);
    double e0 = -theta + (double)i * h, e1 = -theta + (double)(i + 1) * h;
    mass[i] = Phi(((e1 - start) - a) / b) - Phi(((e0 - start) - a) / b);
  }
  for (int n = 0; n < max_steps; ++n) lower[n] = upper[n] = 0.0;
  upper[0] = Phi(-((theta - start) - a) / b);
  lower[0] = Phi(((-theta - start) - a) / b);
  for (int n = 2; n <= max_steps; ++n) {
    double pu = 0.0, pl = 0.0;
    for (int i = 0; i < M; ++i) {
      pu = pu + mass[i] * up[i];
      pl = pl + mass[i] * lo[i];
    }
    upper[n - 1] = pu;
    lower[n - 1] = pl;
    double surv = 0.0;
    for (int j = 0; j < M; ++j) {
      double acc = 0.0;
      for (int i = 0; i < M; ++i) acc = acc + mass[i] * f[j - i + M - 1];
      next[j] = acc;
      surv = surv + acc;
    }
    double *t = mass;
    mass = next;
    next = t;
    if (surv < tol) break;
  }
  free(f); free(up); free(lo); free(mass); free(next);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole sweep                                                               */
/* ------------------------------------------------------------------------ */
int cmo_run(const cmo_model *m, const cmo_sweep *s, cmo_result *r, int n_threads) {
  if (invalid(m, s) || !r || !r->hist || !r->stats) return 1;
  const int64_t S = s->n_settings;
  const uint64_t T = s->trials;
  const int64_t runs = S * (int64_t)T;
  const int width = cmo_state_width(m);
  int8_t *ch = r->run_choice ? r->run_choice : malloc((size_t)runs);
  uint32_t *st = r->run_step ? r->run_step : malloc(sizeof(uint32_t) * (size_t)runs);
  uint8_t *fl = r->run_flag ? r->run_flag : malloc((size_t)runs);
  if (!ch || !st || !fl) return 2;
  rnn_ctx ctx;
  rnn_ctx_init(m, &ctx);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int64_t i = 0; i < runs; ++i) {
    int64_t setting = i / (int64_t)T;
    uint64_t trial = (uint64_t)(i % (int64_t)T);
    double *state = r->run_state ? r->run_state + (size_t)i * width : NULL;
    run_out o = run_one(m, s, &ctx, setting, trial, state, NULL);
    ch[i] = o.choice;
    st[i] = o.steps;
    fl[i] = o.flag;
  }
  rnn_ctx_free(&ctx);

  /* integer reduction into histograms and statistics */
  int32_t correct[9];
  correct_table(m, correct);
  const uint32_t B = s->n_bins, N = s->max_steps;
  memset(r->hist, 0, sizeof(uint64_t) * (size_t)S * 2 * B);
  memset(r->stats, 0, sizeof(uint64_t) * (size_t)S * CMO_NSTAT);
  for (int64_t i = 0; i < runs; ++i) {
    int64_t setting = i / (int64_t)T;
    uint64_t trial = (uint64_t)(i % (int64_t)T);
    uint64_t *stt = r->stats + (size_t)setting * CMO_NSTAT;
    uint64_t n = st[i];
    if (fl[i]) stt[CMO_ST_FLAGGED] += 1;
    if (ch[i] < 0) {
      stt[CMO_ST_UNDEC] += 1;
      continue;
    }
    int c = ch[i];
    uint64_t bin = ((n - 1) * (uint64_t)B) / (uint64_t)N;
    r->hist[((size_t)setting * 2 + (size_t)c) * B + bin] += 1;
    stt[CMO_ST_DEC0 + c] += 1;
    stt[CMO_ST_SUMN0 + c] += n;
    stt[CMO_ST_SUMSQ0 + c] += n * n;
    int stim = (int)(trial % (uint64_t)m->n_stimuli);
    if (correct[stim] == c) stt[CMO_ST_CORRECT] += 1;
  }
  if (!r->run_choice) free(ch);
  if (!r->run_step) free(st);
  if (!r->run_flag) free(fl);

  /* score per setting and the best allocation (random pick among ties) */
  if ((s->reward != 0.0 || s->cost != 0.0) && r->score) {
    double best = -INFINITY;
    for (int64_t i = 0; i < S; ++i) {
      double q = (double)r->stats[(size_t)i * CMO_NSTAT + CMO_ST_CORRECT] / (double)T;
      double pen = 0.0;
      for (int k = 0; k < m->n_signals; ++k) {
        double c = s->grid[i * m->n_signals + k];
        pen = pen + c * c;
      }
      double sc = s->reward * q - s->cost * pen;
      r->score[i] = sc;
      if (sc > best) best = sc;
    }
    if (r->best) {
      int64_t ties = 0, pick = -1;
      uint32_t pick_prio = 0;
      for (int64_t i = 0; i < S; ++i) {
        if (r->score[i] != best) continue;
        ++ties;
        uint32_t w[4];
        uint32_t ctr[4] = {0u, (uint32_t)i, CMO_STREAM_TIE, CMO_STREAM_TIE};
        uint32_t key[2] = {(uint32_t)s->seed, (uint32_t)(s->seed >> 32)};
        cmo_philox4x32_10(ctr, key, w);
        if (pick < 0 || w[0] < pick_prio) { /* settings visited ascending */
          pick = i;
          pick_prio = w[0];
        }
      }
      r->best[0] = pick;
      r->best[1] = ties;
    }
  }
  return 0;
}
