// Internal declarations shared by the libimrt sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "imrt.h"

namespace imrt {

// ---- launch geometry -------------------------------------------------------
constexpr int kThreads = 256;          // 4 wave64 per workgroup
constexpr int kWaves = kThreads / 64;
constexpr int kFwdNnzMax = 2048;       // LDS product slots of one forward row block
constexpr int kFwdPartNnz = kFwdNnzMax - 4;  // block limit so that 16-byte aligned loads fit
constexpr int kFwdRowsMax = 512;       // rows of one forward row block
constexpr int kWaveNnz = 512;          // LDS product slots of one wave's row block (float32 storage)
constexpr int kWavePartNnz = kWaveNnz - 4;
// With 16-bit storage a wave's row block holds twice the nonzeros, so that
// one block's loads are as many bytes as with float32; with float32 values
// and 16-bit column indices it holds 1.5 times as many (6 bytes each).
constexpr int wave_nnz(int storage) { return storage == 0 ? kWaveNnz : storage == 3 ? 3 * kWaveNnz / 2 : 2 * kWaveNnz; }
constexpr int wave_part_nnz(int storage) { return wave_nnz(storage) - 4; }
// Rows of one wave's row block, and the passes of one lane per row over it.
// Every pass's row loads are issued for every block (out-of-range rows read
// zeros), and they cost address cycles even then: fewer passes make the
// blocks of long-row matrices cheaper.
constexpr int kWaveRowsMax = 128;
constexpr int kWavePasses = kWaveRowsMax / 64;
constexpr int kGapRows = 16;           // runs of at least this many empty rows lie between wave blocks
constexpr int kMaxTrials = 4;          // trial step sizes per forward pass
constexpr int kMaxStruct = 256;
constexpr int kPad = 16;               // zeroed tail of every nonzero array (aligned vector loads)
constexpr int kXcds = 8;               // MI355X: 8 accelerator dies, workgroups dealt round-robin
constexpr int64_t kLlcBytes = int64_t(256) << 20;   // MI355X: last-level (Infinity) cache

// ---- device-resident solver state -------------------------------------------
// Phases of the device-side state machine.  Only one workgroup at a time (a
// one-workgroup kernel, or the last workgroup of a pass) writes the state;
// every other kernel reads it at entry and exits early when idle.
enum Phase : int32_t {
  PH_INIT = 0,       // evaluate G(x_1) with the forward pass
  PH_NEED_GRAD = 1,  // gradient of the accepted iterate needed, then a trial pass
  PH_TRIAL = 2,      // the line search needs another trial pass (no new gradient)
  PH_DONE = 3
};

struct SolverState {
  int32_t phase, status, k, m;        // phase, imrt_solve_status, accepted iterations, backtracks
  int32_t acc, xi, n_fwd, n_adj;      // trial whose residual buffer holds r(x_k), iterate buffer of x_k, pass counters
  int32_t ntrials, max_iter, max_bt, fixed;
  int32_t trace_cap, warm;            // trace capacity; warm start of the line search (0/1)
  int32_t resume, pad_;               // resumed solve: G_prev holds G(x_{K-1}) on entry
  double lambda;                      // first trial step of the next forward pass
  double G, G_prev, G_init;
  double eps, alpha, lambda0, delta;
};

struct PenaltyDev {
  double T_u, T_o, w_u, w_o;
};

// Layout-compatible with imrt_trace_entry.
struct TraceDev {
  int32_t k, backtracks;
  double lambda, step_sq, G;
};
static_assert(sizeof(TraceDev) == sizeof(imrt_trace_entry), "trace layout");
static_assert(sizeof(SolverState) % sizeof(int32_t) == 0 && sizeof(SolverState) <= 256 * sizeof(int32_t),
              "state is copied word by word by one workgroup");

// ---- kernel argument blocks ---------------------------------------------------
enum FwdMode : int32_t {
  FWD_SOLVE = 0,  // trials from the solver state; residuals into rbuf; G partials
  FWD_EVAL = 1,   // x given; optional dose and residual outputs; G partials
  FWD_PLAIN = 2   // x given; dose output; partials of sum d^2
};

struct Penalties {
  const uint8_t* sid;        // structure id per voxel
  const PenaltyDev* table;   // per structure
  const float* Tu_vox;       // nullable per-voxel thresholds
  const float* To_vox;
};

// Storage of D's values (the imrt_dtype codes): float32, or 16-bit codes q
// with a float32 scale per beamlet (D~_ij = col_scale[i] * q_ij), where the
// CSR column indices are 16-bit too.
enum Storage : int32_t { ST_F32 = 0, ST_BF16 = 1, ST_F16 = 2 };
// Layout the forward pass reads: the storage's own, or for float32 values
// with nb <= 65536 the CSR column indices as 16 bits (ST_F32C16).  The
// arithmetic is that of float32 storage.
constexpr int32_t ST_F32C16 = 3;
constexpr bool coded(int st) { return st == ST_BF16 || st == ST_F16; }

struct FwdArgs {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const float* val;
  const uint16_t* col16;     // 16-bit storage or ST_F32C16: column indices
  const uint16_t* val16;     // 16-bit storage: codes
  const float* col_scale;    // 16-bit storage: per-beamlet scale (else null)
  int32_t storage;
  int32_t waves;             // waves of a wave-granular forward workgroup (8 or 16; 8 with four trials)
  int32_t stream_cp;         // host side: cache policy of a solve pass's matrix streams (0 or 2)
  const int32_t* block_row;  // nblocks + 1 row boundaries
  const int32_t* block_k0;   // nblocks + 1 nonzero offsets of the blocks
  int32_t nblocks, nv, nb, mode;
  const int32_t* wblock_row; // per-wave row blocks (wave-granular forward): first row,
  const int32_t* wblock_k0;  // first nonzero (block b ends at wblock_k0[b + 1]),
  const int32_t* wblock_end; // end row (runs of empty rows between blocks are skipped)
  int32_t nwblocks;
  int32_t grid;              // workgroups of this pass (read by the batched pass)
  int32_t nstruct;
  Penalties pen;
  const float* x;            // eval/plain input vector
  // solve: gradient of x_k (complete for columns of one adjoint workgroup;
  // shared columns from their pieces), iterate buffers, residual buffers
  const float* g;
  const uint8_t* col_kind;   // 0: one adjoint workgroup, 1: two (pieces_col), 2: more (pieces)
  const double* pieces_col;
  const double* pieces;
  const int32_t* col_wlo;
  const int32_t* col_whi;
  double g_scale;
  float* xbuf[kMaxTrials + 1];  // x_k = xbuf[st->xi]; trial q goes to xbuf[(xi + 1 + q) % (NT + 1)]
  float* rbuf[kMaxTrials + 1];  // residual of trial q into rbuf[q] (r(x_k) = rbuf[st->acc])
  float* d_out;              // eval/plain: dose (nullable in eval)
  float* r_out;              // eval: residual (nullable)
  double* partials;          // [trial][gridDim.x] objective partials, then (solve) [trial] step norms
  const SolverState* st_in;  // solve: state before this pass
  SolverState* st_out;       // solve: state after it (copied through by workgroup 0)
};

// Adjoint work partition: workgroup w owns nonzeros [w*nnz/G, (w+1)*nnz/G)
// of the CSC arrays, i.e. columns [c0, c1) in part or whole, where
// wg_cols[4w..4w+3] = {c0, c1, lo, hi} and [lo, hi) is the part of column c0
// inside the range (c0 = c1 = lo = hi = 0 without columns).
// Column c is shared by workgroups col_wlo[c]..col_whi[c]; a shared column is
// completed from the per-workgroup pieces (slot 2w: piece of w's first
// column, slot 2w+1: piece of its last column) in workgroup order.
struct AdjArgs {
  const int32_t* row_idx;
  const float* val;
  const uint16_t* val16;     // 16-bit storage: codes (CSC slot order)
  const float* col_scale;    // 16-bit storage: per-beamlet scale (else null)
  int32_t storage;
  int32_t stream_cp;         // host side: cache policy of a solve pass's matrix streams (0 or 2)
  const int32_t* col_ptr;
  const int32_t* wg_cols;
  const int32_t* col_wlo;
  const int32_t* col_whi;
  const uint8_t* col_kind;   // 0: one adjoint workgroup, 1: two, 2: more
  int64_t nnz;
  int32_t nv, nb, grid;
  int32_t xcd_map;           // workgroup ranges contiguous per accelerator die (else dispatch order)
  int32_t solve;             // decide the previous forward pass first; r from rbuf
  const float* r;
  float* rbuf[kMaxTrials + 1];
  double* pieces;            // 2 * grid
  double* pieces_col;        // nullable, 2 * nb: pieces of columns shared by two workgroups, by column
  float* out;
  double scale;
  // solve: line-search decision on the previous forward pass
  const double* fwd_partials;   // [trial][fwd_parts]
  int32_t fwd_parts;
  const double* step_partials;  // [trial][step_parts] step norms ||x_t - x_k||^2
  int32_t step_parts;
  const SolverState* st_in;
  SolverState* st_out;
  TraceDev* trace;
  double G_skip;             // objective of the voxels the wave forward skips (rows without
                             // nonzeros between its blocks), added to every trial's G
};

// ---- host-side objects ------------------------------------------------------------
struct Tuning {
  int fwd_grid_per_cu = 3;
  int adj_grid_per_cu = 4;
  int adj_min_nnz = 1024;      // nonzeros per adjoint workgroup at least (small matrices)
  int batch_iters = 32;        // iterations enqueued between host polls
  int voxel_tiles = 1;         // built phantoms: voxels in 4x4x2 tiles (1) or the grid's own order (0)
  int adj_xcd = 1;             // adjoint ranges contiguous per accelerator die (1) or in dispatch order (0)
  int fwd_wave = 1;            // forward rows blocks per wave (1) or per workgroup (0)
  int fwd_bpw = 1;             // fewest row blocks per forward wave (new dose matrices)
  int fwd_col16 = 1;           // float32 matrices with nb <= 65536: 16-bit CSR columns for the forward
  int part_adj_wgs = 0;            // > 0: new matrices take the per-plan partition targets
  int part_fwd_wgs = 0;            // (adjoint / forward workgroups) instead of the two above
  int serve_adj_wgs = 128;         // the targets of the matrices a server builds, which
  int serve_fwd_wgs = 32;          // share their dispatches with the other live plans
  int serve_groups = 16;           // (adjoint, forward) groups a server runs between polls
  int serve_shared_adj = 0;        // live solves on one resident matrix share its adjoint pass
  int stream_nt = 2;               // solve passes read the matrix streams non-temporally: 0 never,
                                   // 1 always, 2 when they exceed the last-level cache
};

}  // namespace imrt

struct imrt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  size_t max_lds = 65536;
  size_t cu_lds = 65536;   // LDS of one compute unit (workgroups that fit side by side)
  imrt::Tuning tune;
};

struct imrt_dose {
  imrt_ctx* ctx = nullptr;
  int device = 0;
  int32_t nv = 0, nb = 0;
  int64_t nnz = 0;
  // CSR (forward) and CSC (adjoint) copies of D, each nonzero array padded by kPad zeros
  int32_t* row_ptr = nullptr;
  int32_t* col_idx = nullptr;
  float* val = nullptr;
  int32_t* col_ptr = nullptr;
  int32_t* row_idx = nullptr;
  float* cval = nullptr;
  // 16-bit storage (then col_idx, val and cval are released): CSR column
  // indices and codes, CSC codes, per-beamlet scales
  int32_t storage = 0;
  int32_t fwd_st = -1;         // the forward layout (Storage or ST_F32C16), set with the partition
  uint16_t* col16 = nullptr;   // (also kept beside col_idx for ST_F32C16)
  uint16_t* val16 = nullptr;
  uint16_t* cval16 = nullptr;
  float* col_scale = nullptr;
  // work partitions: fewest nonzeros per adjoint workgroup and row blocks
  // per forward wave (from the context's options when created; changed by
  // imrt_dose_repartition)
  int32_t adj_min_nnz = 1024, fwd_bpw = 1;
  // Waves of a forward workgroup with one or two trials per pass: 16 (one
  // workgroup per compute unit) for a matrix solved alone, 8 (three side by
  // side) once per-plan targets are applied for shared dispatches.
  int32_t fwd_waves = 16;
  // forward row blocks and adjoint chunks
  int32_t nblocks = 0;
  int32_t* block_row = nullptr;
  int32_t* block_k0 = nullptr;
  int32_t nwblocks = 0;
  int32_t* wblock_row = nullptr;
  int32_t* wblock_k0 = nullptr;
  int32_t* wblock_end = nullptr;
  // runs of empty rows the wave blocks skip, [first, end) in internal row
  // order, and a counter of partitions (a plan's constant for the skipped
  // rows follows it)
  std::vector<std::pair<int32_t, int32_t>> gaps;
  int64_t part_epoch = 0;
  int32_t adj_grid = 0;        // workgroups of the adjoint partition
  int32_t* wg_cols = nullptr;
  int32_t* col_wlo = nullptr;
  int32_t* col_whi = nullptr;
  uint8_t* col_kind = nullptr; // per column: 0 one adjoint workgroup, 1 two, 2 more
  double* pieces = nullptr;
  // internal voxel order (nullable: the caller's order): row p of D is voxel
  // vox[p]; every voxel-indexed array crossing the API is permuted
  int32_t* vox = nullptr;
  std::vector<int32_t> vox_host;
  float* vscratch = nullptr;   // nv floats for permuted products
  // structure ids from the phantom builder (nullable; internal order)
  uint8_t* sid = nullptr;
  // scratch for plain products
  double* partials = nullptr;
  int32_t partials_len = 0;
  int32_t fwd_cap = 1;         // forward grids are capped at the partials capacity
};

struct imrt_plan {
  imrt_ctx* ctx = nullptr;
  int device = 0;
  const imrt_dose* dose = nullptr;
  uint8_t* sid = nullptr;
  int32_t nstruct = 0;
  bool have_struct = false, have_pen = false;
  imrt::PenaltyDev* table = nullptr;
  double w_max = 0.0;
  float* Tu_vox = nullptr;
  float* To_vox = nullptr;
  // workspace
  float* rbuf[imrt::kMaxTrials + 1] = {};
  float* xbuf[imrt::kMaxTrials + 1] = {};
  float* gk = nullptr;
  float* vtmp = nullptr;          // nv scratch
  double* fwd_partials = nullptr; // kMaxTrials * (fwd_cap + 1)
  int32_t fwd_cap = 1;
  double* pieces = nullptr;       // 2 * adjoint grid
  int32_t pieces_cap = 0;         // adjoint grid the pieces were sized for
  double* pieces_col = nullptr;   // 2 * nb
  double* misc = nullptr;         // small reduction scratch
  imrt::SolverState* st = nullptr;  // 2 states, alternately read and written by consecutive passes
  imrt::TraceDev* trace = nullptr;
  int32_t trace_cap = 0;
  imrt::SolverState* st_host = nullptr;   // pinned, 2 slots
  double* misc_host = nullptr;            // pinned
  // host copies (internal voxel order) for the objective of the voxels the
  // wave forward skips: structure ids, penalty table, per-voxel targets
  std::vector<uint8_t> sid_host;
  std::vector<imrt::PenaltyDev> table_host;
  std::vector<float> Tu_host, To_host;
  double G_skip = 0.0;
  int64_t gskip_epoch = -1;               // dose partition the constant was computed for (-1: stale)
  std::vector<int64_t> skip_hist;         // skipped rows per structure id
  int64_t skip_hist_epoch = -1;
};

namespace imrt {

// error reporting (thread-local message)
int set_error(int code, const std::string& msg);
int hip_error(hipError_t e, const char* what);

#define IMRT_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return imrt::hip_error(e_, #call); \
  } while (0)

// launchers (kernels.hip)
// forward grid: wave-granular pass, fwd_grid_per_cu workgroups of 16 waves
// (8 for several trials) per CU; workgroup-granular pass, 4x as many of 4 waves
int forward_grid(const imrt_ctx* ctx, const imrt_dose* D, int ntrials = 1);
int wave_grid(const imrt_ctx* ctx, int nwblocks, int ntrials, int blocks_per_wave, int nb, int storage,
              int dose_waves);
int forward_waves(int ntrials, int dose_waves);
int adjoint_grid_for(const imrt_ctx* ctx, int64_t nnz, int min_nnz);
size_t forward_lds_bytes(int nb, int ntrials, int nstruct, bool wave, int storage, int dose_waves);
__host__ __device__ inline int pad4(int n) { return (n + 3) & ~3; }

// CSC nonzero k is stored at slot csc_slot(k): within every aligned tile of
// 256 entries, entry 64u + i (i < 64, u < 4) sits at 4i + u, so one 16-byte
// load by lane i brings entries i, i + 64, i + 128, i + 192 of its tile and
// each of the four components is a run of 64 consecutive entries across the
// wave (consecutive rows of a column: their residual gathers coalesce).
constexpr int kTile = 256;
__host__ __device__ inline int64_t csc_slot(int64_t k) {
  return (k & ~static_cast<int64_t>(kTile - 1)) | ((k & 63) << 2) | ((k >> 6) & 3);
}
__host__ __device__ inline int64_t csc_entry(int64_t slot) {
  return (slot & ~static_cast<int64_t>(kTile - 1)) | ((slot & 3) << 6) | ((slot >> 2) & 63);
}
// Entries allocated for the CSC arrays of nnz nonzeros (whole tiles plus one).
inline size_t csc_alloc(int64_t nnz) { return static_cast<size_t>(((nnz + kTile - 1) / kTile + 1) * kTile); }
int launch_forward(const imrt_ctx* ctx, const imrt_dose* D, const FwdArgs& a, int ntrials, int grid,
                   hipEvent_t before = nullptr, hipEvent_t after = nullptr);
int launch_adjoint(const imrt_ctx* ctx, const imrt_dose* D, const AdjArgs& a, int ntrials,
                   hipEvent_t before = nullptr, hipEvent_t after = nullptr);
// Batched solve passes over a slot table (device arrays of per-plan arguments
// and of (plan << 16 | workgroup) slots, -1 for an idle slot).
// stream_cp: cache policy of the matrix streams (0 default, 2 non-temporal).
int launch_forward_batch(const imrt_ctx* ctx, const FwdArgs* args, const int32_t* slots, int nslots, int ntrials,
                         int storage, int dose_waves, size_t lds, int stream_cp);
int launch_adjoint_batch(const imrt_ctx* ctx, const AdjArgs* args, const int32_t* slots, int nslots, int ntrials,
                         int storage, int stream_cp);
// Adjoint passes of groups of solves sharing a dose matrix: groups[(K + 1) g]
// = n <= K, then n plan indices into args; slots = (group << 16) | workgroup.
// group_k (K) is 2 or 4.
int launch_adjoint_multi_batch(const imrt_ctx* ctx, const AdjArgs* args, const int32_t* groups, int group_k,
                               const int32_t* slots, int nslots, int ntrials, int storage);
// out = (fixed-order sum of parts[0..n)) + add
int launch_sum(const imrt_ctx* ctx, const double* parts, int n, double* out, double add = 0.0);
// p[0..n) = 0 with a kernel (usable under graph capture, unlike a memset node)
int launch_zero(const imrt_ctx* ctx, float* p, int n);
int launch_project(const imrt_ctx* ctx, const float* x, const float* g, double lambda, int nb,
                   float* x_out, double* s_out);
int launch_normalize(const imrt_ctx* ctx, const float* w, int nb, float* v_out, double* norm_out);
// out[vox[p]] = in[p] (scatter) or out[p] = in[vox[p]] (gather), p < n
int launch_permute(const imrt_ctx* ctx, const float* in, const int32_t* vox, int n, float* out, bool scatter);
// Replace D's float32 values by 16-bit codes with per-beamlet scales (build.hip).
int store16(imrt_dose* D, int storage);

// phantom builder (build.hip)
int build_phantom(imrt_ctx* ctx, const imrt_geometry* g, imrt_dose* D);
// Partition of a matrix of nnz nonzeros for about `ta` adjoint and `tf`
// forward workgroups: nonzeros per adjoint workgroup in [1024, 32768], row
// blocks per forward wave in [1, 4].
void partition_for_targets(int64_t nnz, int ta, int tf, int32_t* adj_min_nnz, int32_t* fwd_bpw);
// The context's per-plan targets (if set) fixed as D's partition, once nnz is known.
void apply_partition_targets(const imrt_ctx* ctx, imrt_dose* D);

// host preprocessing (api.hip)
int alloc_nonzeros(imrt_dose* D);
int finish_dose(imrt_dose* D, const std::vector<int32_t>& row_ptr, const std::vector<int32_t>& col_ptr);

}  // namespace imrt
