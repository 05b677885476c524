/*
 * cmo.h -- plain FP64 CPU oracle for batched cognitive-model simulation.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the HIP path
 * against a slow, obviously correct implementation.  No product code may
 * load or call it.  It shares no code, header, table or constant with the
 * HIP library: everything here is written out on its own from the method's
 * definition (the Distill paper, Sec. 2.2 "Cognitive Model Execution" and its
 * scheduling listing, Sec. 3.3 "Dynamic to Static Data Structure Conversion",
 * Sec. 3.6 "Parallelism and GPU Acceleration", Sec. 4.4 "Clone detection"
 * for the DDM/LCA mechanisms) plus readings, stated where they are used,
 * for what the paper leaves open.
 *
 * All pointers are HOST pointers.  The caller owns every buffer; outputs are
 * fully overwritten (histograms and statistics are zeroed first).
 */
#ifndef CMO_H
#define CMO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* model kinds */
enum { CMO_DDM = 0, CMO_LCA = 1, CMO_RNN = 2, CMO_LOOP = 3 };
/* precision modes */
enum { CMO_FP64 = 0, CMO_FP32_STEP = 1, CMO_BF16_PROJ = 2 };

/* Parameter slots: string keys become fixed offsets (Sec. 3.3). */
enum { CMO_DDM_DT = 0, CMO_DDM_DRIFT, CMO_DDM_NOISE, CMO_DDM_THRESH,
       CMO_DDM_START, CMO_DDM_T0, CMO_DDM_NPARAM };
enum { CMO_LCA_DT = 0, CMO_LCA_LEAK, CMO_LCA_COMP, CMO_LCA_NOISE,
       CMO_LCA_THRESH, CMO_LCA_OFFSET, CMO_LCA_HID_GAIN, CMO_LCA_HID_BIAS,
       CMO_LCA_NONNEG, CMO_LCA_T0, CMO_LCA_NPARAM };
enum { CMO_RNN_DT = 0, CMO_RNN_NOISE, CMO_RNN_THRESH, CMO_RNN_INPUT_GAIN,
       CMO_RNN_T0, CMO_RNN_NPARAM };
/* Closed-loop control of the conflict network: the LCA parameters, then the
 * control search (levels per signal L, top level A_max, look-ahead samples M,
 * control-cost weight). */
enum { CMO_LOOP_LEVELS = CMO_LCA_NPARAM, CMO_LOOP_AMAX, CMO_LOOP_SAMPLES, CMO_LOOP_COST,
       CMO_LOOP_NPARAM };

/* statistics per setting */
enum { CMO_ST_DEC0 = 0, CMO_ST_DEC1, CMO_ST_UNDEC, CMO_ST_CORRECT,
       CMO_ST_SUMN0, CMO_ST_SUMN1, CMO_ST_SUMSQ0, CMO_ST_SUMSQ1,
       CMO_ST_FLAGGED, CMO_NSTAT };

/* Random stream ids (counter word 3). */
#define CMO_STREAM_DRIVE 0x40000000u
#define CMO_STREAM_TIE 0xFFFFFFFFu
#define CMO_STREAM_LOOK 0x80000000u /* | (allocation * M + sample), < 2^30 */
#define CMO_STREAM_PICK 0xC0000000u /* | allocation */

typedef struct {
  int32_t kind, precision;
  int32_t n_units;     /* DDM 1, LCA 2, RNN n (even, <= 1024), LOOP 2 */
  int32_t n_stimuli;   /* DDM 1, LCA 9, RNN 1 */
  int32_t n_signals;   /* DDM 0/1 (drift), LCA 0/2 (cA,cB), RNN 0/1 (gain) */
  const double *params;
  int32_t n_params;
  const double *weights; /* LCA: WA[4x3] WB[4x3] OA[2x4] OB[2x4]; RNN: W[nxn] R[2xn] */
  int64_t n_weights;
} cmo_model;

typedef struct {
  const double *grid;  /* [n_settings x n_signals] or NULL when n_signals==0 */
  int64_t n_settings;
  uint64_t trials;     /* per setting */
  uint64_t seed;
  uint32_t max_steps, n_bins;
  double reward, cost; /* both 0: no score */
  double flag_eps;
} cmo_sweep;

typedef struct {
  uint64_t *hist;     /* [n_settings][2][n_bins] */
  uint64_t *stats;    /* [n_settings][CMO_NSTAT] */
  double *score;      /* [n_settings] or NULL */
  int64_t *best;      /* [2] or NULL */
  int8_t *run_choice; /* optional per-run dumps, [n_settings*trials] */
  uint32_t *run_step;
  uint8_t *run_flag;
  double *run_state;  /* [runs][state width]: DDM 1, LCA 2, RNN 2+n */
} cmo_result;

/* Whole sweep.  Returns 0 on success, nonzero on invalid arguments. */
int cmo_run(const cmo_model *m, const cmo_sweep *s, cmo_result *r, int n_threads);

/* Building blocks exposed for pins. */
void cmo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void cmo_normals64(const uint32_t w[4], double z[2]);
void cmo_normals32(const uint32_t w[4], float z[2]);
double cmo_ddm_update(double x, double a, double b, double z);
void cmo_lca_update(const double x[2], const double in[2], double leak, double comp,
                    double dt, double b, const double z[2], double out[2]);
/* conflict-network drive I[stim][2] and correct response per stimulus */
void cmo_conflict_drive(const double *weights, double gain, double bias, double offset,
                        double cA, double cB, double drive[9][2]);
void cmo_conflict_correct(const double *weights, double gain, double bias, int32_t correct[9]);
/* one run's trajectory: state after each executed step, [steps][width];
 * returns the number of executed steps, writes choice and flag. */
uint32_t cmo_trajectory(const cmo_model *m, const cmo_sweep *s, int64_t setting,
                        uint64_t trial, double *states, int8_t *choice, uint8_t *flag);
/* First-passage probabilities of the discretised DDM x_n = x_{n-1} + a + b z
 * with bounds +-theta, by density propagation on `cells` cells; lower[n-1]
 * and upper[n-1] receive the probability of a decision at step n.  Stops
 * once the survivor mass falls below tol (remaining entries 0). */
int cmo_ddm_density(double a, double b, double theta, double start, int cells, int max_steps,
                    double tol, double *lower, double *upper);
/* Time course of the ensemble: at every sample step n = every*k (k = 1..K,
 * K = max_steps / every) the runs of each setting that executed step n (their
 * decision step is n or later) contribute their state after step n.
 * tc[(setting*K + k-1)*CMO_TC_WORDS + c] receives, for c =
 *   0 count of contributing runs,
 *   1 sum q(x0), 2 sum q(x1), 3 sum q(x0*x0), 4 sum q(x1*x1),
 *   5 sum q(comp*(x0*x1)) (the response layer's conflict energy),
 * with q(v) = v*2^32 rounded to nearest (ties to even), clamped to +-2^62,
 * and two's-complement (mod 2^64) sums.  The DDM has x1 = 0 (words 2, 4 and
 * 5 stay 0).  DDM and conflict LCA only.  Returns 0 on success. */
#define CMO_TC_WORDS 6
int cmo_timecourse(const cmo_model *m, const cmo_sweep *s, uint32_t every, int64_t *tc,
                   int n_threads);
/* the quantisation above, for pins */
int64_t cmo_tc_quant(double v);

/* round-to-nearest-even double -> float -> bfloat16 bits */
uint16_t cmo_bf16_bits(double v);
int cmo_state_width(const cmo_model *m);

#ifdef __cplusplus
}
#endif
#endif
