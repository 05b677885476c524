// internal.hpp -- host/device declarations shared by libcm's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cm.h"
#include "lca_step.hpp"

namespace cm {

// Per-setting record of the LDS histogram window, in 32-bit words:
// hist[2][B] counts, 8 count words (dec0, dec1, undec, correct, flagged, pad),
// then 4 uint64 sums (sum n for choice 0/1, sum n^2 for choice 0/1).
enum { kCntDec0 = 0, kCntDec1, kCntUndec, kCntCorrect, kCntFlagged, kCntWords = 8 };
__host__ __device__ inline uint32_t rec_words(uint32_t n_bins) { return 2u * n_bins + kCntWords + 8u; }
// Time-course block per setting: K samples x kTcWords 64-bit sums (count,
// x0, x1, x0^2, x1^2, energy), in 32-bit words.
constexpr uint32_t kTcWords = 6;
__host__ __device__ inline uint32_t tc_words(uint32_t k) { return 2u * kTcWords * k; }

// Arguments of the lane-per-run simulation kernels (DDM, conflict LCA).
struct SimArgs {
  uint64_t trials, n_settings, total_runs, seed;
  uint64_t chunk;     // runs handed to one workgroup
  uint32_t max_steps, n_bins, n_signals, window, steps_per_sync;
  double thresh, flag_eps, b, dt;
  double drift, start;  // DDM
  double leak, comp;    // LCA
  LcaF32 pf;            // LCA, FP32 steps: float(leak dt), float(comp dt), float(b)
  float bf;             // float(b)
  float guard_f;        // float(thresh - 2 flag_eps)
  uint32_t nonneg;
  uint32_t direct;  // 1: count finished runs straight into global memory
  uint64_t trials_magic, steps_magic;  // udiv_magic multipliers for trials and max_steps
  int64_t* tc;                         // time course [n_settings][tc_k][kTcWords] or NULL
  uint32_t tc_every, tc_k;
  const double* grid;
  const double* drive;     // LCA: [settings][9][2]
  const int32_t* correct;  // [stimuli]
  uint64_t* hist;
  uint64_t* stats;
  int8_t* run_choice;
  uint32_t* run_step;
  uint8_t* run_flag;
  double* run_state;
};

// Quotient n / d of 32-bit values by one 64x32 multiply-high, with
// M = floor((2^64 - 1) / d) + 1 (0 for d = 1).  Exact for every n < 2^32:
// M = (2^64 + e) / d with 0 <= e <= d, so n M / 2^64 exceeds n / d by less
// than 2^-32, less than the gap 1/d between n / d and the next integer.
__host__ __device__ inline uint64_t udiv_magic_for(uint32_t d) {
  return d == 1u ? 0ull : ~0ull / d + 1ull;
}
__host__ __device__ inline uint32_t udiv_magic(uint32_t n, uint64_t M) {
  if (M == 0) return n;
  const uint64_t lo = (uint64_t)n * (uint32_t)M;
  const uint64_t hi = (uint64_t)n * (uint32_t)(M >> 32) + (lo >> 32);
  return (uint32_t)(hi >> 32);
}

// Up to kMaxBatch sweeps of one kind and precision in one launch.
constexpr uint32_t kMaxBatch = 12;
struct LaneBatch {
  uint32_t n;
  uint32_t pad;
  uint64_t base[kMaxBatch + 1];  // first workgroup of each sweep; base[n] = grid size
  SimArgs a[kMaxBatch];
};

struct ScoreArgs {
  uint64_t n_settings, trials, seed;
  uint32_t n_signals;
  double reward, cost;
  const double* grid;
  const uint64_t* stats;
  double* score;
  int64_t* best;
};

struct DriveArgs {
  uint64_t n_settings;  // rows of the drive table (allocations in the closed loop)
  uint32_t n_signals;
  uint32_t levels;      // closed loop: row j is allocation (level j / L, level j % L)
  double amax;          // closed loop: top control level
  double gain, bias, offset;
  const double* weights;
  const double* grid;
  double* drive;     // [settings][9][2]
  int32_t* correct;  // [9]
  double* norm2;     // closed loop: [allocations] c_A^2 + c_B^2, else NULL
};

// Per-sweep preparation, many sweeps per launch: zero the histogram and
// statistics (and the time course), then write the correct-response table
// (and, for the conflict network, the drive table).  Item k covers launch indices [end[k-1], end[k]).
struct PrepItem {
  uint64_t* hist;
  uint64_t n_hist;
  uint64_t* stats;
  uint64_t n_stats;
  uint64_t* extra;  // a third range to zero (the time course) or NULL
  uint64_t n_extra;
  uint32_t kind;  // CM_DDM: correct[0] = 1; CM_CONFLICT_LCA: drive and correct; else none
  uint32_t pad;
  DriveArgs d;  // d.correct for the DDM and the conflict network; the rest for the latter
  uint64_t end;
};
struct PrepBatch {
  uint32_t n;
  uint32_t pad;
  PrepItem it[kMaxBatch];
};
struct ScoreBatch {
  uint32_t n;
  uint32_t pad;
  ScoreArgs a[kMaxBatch];
};

// Device work queue of the serving path: a persistent lane kernel takes
// requests that the host publishes in pinned host memory, each as (slot,
// item count) in a ring and a descriptor per slot.  A request's items are its
// preparation pieces (zero-fill and tables) and then its chunks, each run as
// one workgroup of the batched kernel would run it; the chunks wait for the
// preparation, and the workgroup that finishes the last chunk scores the
// sweep (when it is scored) and marks the request done.  One workgroup at a
// time copies newly published ring entries and their descriptors into
// device memory, so host memory is read once per request.  Workgroups claim
// items with one fetch-and-add on a 64-bit word holding (request index, next
// item); the word moves to the next request by compare-and-swap only once
// every item of the current one is claimed.
constexpr uint64_t kQueuePrepSpan = 1u << 12;  // preparation indices per piece
struct QueueReq {
  // (publication number << 32) | item count, read and written as one word:
  // the number tells a stale entry from the one that replaced it
  unsigned long long num_items;
  uint32_t slot, pad;
};
struct QueueDesc {
  SimArgs a;
  PrepItem prep;
  ScoreArgs score;
  uint64_t prep_target;   // the slot's preparation pieces once this request's are done
  uint64_t chunk_target;  // the slot's chunks once this request's are done
  uint32_t pieces;        // items [0, pieces) are preparation pieces, the rest chunks
  uint32_t ticket;        // low 32 bits of the request's ticket, stored in done[slot] at the end
  uint32_t scored;
  uint32_t pad;
};
static_assert(sizeof(QueueDesc) % 8 == 0, "descriptors are copied in 8-byte words");
struct QueueArgs {
  const uint32_t* tail;   // HOST: requests published so far
  const uint32_t* stop;   // HOST: non-zero ends the kernel
  uint32_t* done;         // HOST [slots]: ticket of the slot's last finished request
  const QueueReq* ring;   // HOST [cap_ring]: request i at i % cap_ring
  const QueueDesc* desc;  // HOST [slots]
  uint32_t cap_ring;
  uint32_t pad;
  unsigned long long* word;  // DEVICE: (request index << 32) | next item of that request
  uint32_t* dev_tail;        // DEVICE: requests copied to the device so far (<= *tail)
  uint32_t* pull_lock;       // DEVICE: 1 while one workgroup reads the host's queue
  uint32_t* dev_stop;        // DEVICE: the host's stop flag, as last read
  QueueReq* dring;           // DEVICE [cap_ring]: copies of the host's ring
  QueueDesc* ddesc;          // DEVICE [slots]: copies of the host's descriptors
  unsigned long long* prep_done;   // DEVICE [slots]: preparation pieces finished, cumulative
  unsigned long long* chunk_done;  // DEVICE [slots]: chunks finished, cumulative
  uint64_t idle_ticks;             // real-time clock ticks without an item before exiting
};

// Arguments of the rate-network kernels.
struct RnnArgs {
  uint64_t trials, n_settings, total_runs, seed;
  uint32_t max_steps, n_bins, n_signals, n_units;
  double thresh, flag_eps, b, dt, gain;
  const double* grid;
  const void* wfrag;  // W in matrix-core fragment order (bf16 or fp64)
  const double* R;    // readout weights [2][n]
  uint64_t* hist;
  uint64_t* stats;
  int8_t* run_choice;
  uint32_t* run_step;
  uint8_t* run_flag;
  double* run_state;
};

// Arguments of the node-by-node (unfused) execution.
struct UnfusedArgs {
  uint64_t trials, n_settings, total_runs, seed;
  uint32_t max_steps, n_bins, n_signals, kind;
  double thresh, flag_eps, b, dt, drift, start, leak, comp;
  uint32_t nonneg;
  const double* grid;
  const double* drive;
  const int32_t* correct;
  double* x;       // [runs][2]
  double* z;       // [runs][2]
  uint32_t* n;     // [runs]
  uint8_t* flag;   // [runs]
  int8_t* choice;  // [runs]
  uint32_t* active;  // [2][runs]
  uint32_t* count;   // [2]
  uint64_t* hist;
  uint64_t* stats;
  int8_t* run_choice;
  uint32_t* run_step;
  uint8_t* run_flag;
  double* run_state;
};

// Arguments of the closed-loop control kernel.
struct LoopArgs {
  uint64_t trials, n_settings, total_runs, seed;
  uint64_t steps_magic;
  uint32_t max_steps, n_bins, n_signals, L, J, M, nonneg, pad;
  double thresh, flag_eps, b, dt, leak, comp, cost;
  const double* grid;      // [n_settings] control-cost weights, or NULL
  const double* drive;     // [J][9][2]
  const double* norm2;     // [J] c_A^2 + c_B^2 of allocation j
  const int32_t* correct;  // [9]
  uint64_t* hist;
  uint64_t* stats;
  int8_t* run_choice;
  uint32_t* run_step;
  uint8_t* run_flag;
  double* run_state;
};

// Arguments of the DDM density propagation.
struct DensityArgs {
  uint64_t n_settings;
  uint32_t max_steps, cells, n_signals;
  double dt, drift, b, thresh, start, tol;
  const double* grid;
  double* out;  // [settings][2][max_steps]
};

// Launchers (return the hipError_t of the launch).
// scan_block: 0 for the lane kernel, else the DDM scan kernel with that many
// threads (256 or 512) per workgroup.
// occ: 0, or 4 / 8 for the lane kernel built with registers capped so that
// that many wavefronts fit per SIMD (ignored by the scan kernel).
// block: threads per workgroup of the lane kernel, 256, 512 or 1024 (256
// for the time-course variant; ignored by the scan kernel).
hipError_t launch_sim_lane(int kind, int precision, uint32_t scan_block, bool tc, uint32_t occ,
                           uint32_t block, const LaneBatch& b, size_t lds_bytes, hipStream_t st);
hipError_t launch_prep(const PrepBatch& b, hipStream_t st);
hipError_t launch_ceiling(int kind, int precision, const SimArgs& a, uint32_t steps, uint64_t lanes,
                          double* out, hipStream_t st);
// The persistent queue kernel of kind/precision (conflict LCA) on `groups`
// workgroups of 256 threads with lds_bytes of dynamic LDS.
hipError_t launch_queue(int kind, int precision, const QueueArgs& q, uint32_t groups, size_t lds_bytes,
                        hipStream_t st);
// LDS after the histogram window (and the time-course blocks) that the lane
// kernel uses to pack unfinished runs while a chunk drains.
size_t lane_stage_bytes(int kind, int precision, uint32_t block);
hipError_t launch_score(const ScoreBatch& b, hipStream_t st);
uint32_t loop_team_lanes(uint32_t J, uint64_t runs, uint32_t cus);
hipError_t launch_loop(int precision, const LoopArgs& a, uint32_t team, uint32_t blocks, hipStream_t st);
hipError_t launch_rnn_prep(const double* W, uint32_t n, void* out, bool bf16, hipStream_t st);
hipError_t launch_rnn(int precision, const RnnArgs& a, uint32_t groups, hipStream_t st);
hipError_t launch_uf_init(const UnfusedArgs& a, hipStream_t st);
hipError_t launch_uf_step(const UnfusedArgs& a, int precision, uint32_t n, int cur, uint64_t bound,
                          hipStream_t st);
hipError_t launch_uf_reduce(const UnfusedArgs& a, hipStream_t st);
hipError_t launch_ddm_density(const DensityArgs& a, hipStream_t st);
size_t density_lds_bytes(uint32_t cells);

}  // namespace cm
