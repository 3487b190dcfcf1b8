// Internal declarations shared by the libimrt sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "imrt.h"

namespace imrt {

// ---- launch geometry -------------------------------------------------------
constexpr int kThreads = 256;          // 4 wave64 per workgroup
constexpr int kWaves = kThreads / 64;
constexpr int kFwdNnzMax = 2048;       // nonzeros of one forward row block (staged in LDS)
constexpr int kFwdRowsMax = 512;       // rows of one forward row block
constexpr int kAdjChunk = 2048;        // target nonzeros of one adjoint work item
constexpr int kMaxTrials = 4;          // trial step sizes per forward pass
constexpr int kMaxStruct = 256;

// ---- device-resident solver state -------------------------------------------
// Phases of the device-side state machine.  Only single-workgroup kernels (or
// the last workgroup of a kernel) write the state; every other kernel reads it
// at entry and exits early when there is nothing to do.
enum Phase : int32_t {
  PH_INIT = 0,       // evaluate G(x_1) with the forward pass
  PH_NEED_GRAD = 1,  // gradient of the accepted iterate needed, then a trial pass
  PH_TRIAL = 2,      // the line search needs another trial pass (no new gradient)
  PH_DONE = 3
};

struct SolverState {
  int32_t phase, status, k, m;        // phase, imrt_solve_status, accepted iterations, backtracks
  int32_t acc, n_fwd, n_adj, ntrials; // residual buffer of x_k, pass counters, trials per pass
  int32_t max_iter, max_bt, fixed, trace_cap;
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

struct FwdArgs {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const float* val;
  const int32_t* block_row;  // nblocks + 1 row boundaries
  int32_t nblocks, nv, nb, mode;
  Penalties pen;
  const float* x;            // x_k (solve) or the input vector
  const float* g;            // g_k (solve)
  float* rbuf[kMaxTrials + 1];
  float* d_out;              // eval/plain: dose (nullable in eval)
  float* r_out;              // eval: residual (nullable)
  double* partials;          // [trial][gridDim.x]
  SolverState* st;
};

struct AdjArgs {
  const int32_t* row_idx;
  const float* val;
  const int32_t* chunk_k;    // nchunks + 1 nonzero boundaries (each chunk inside one column)
  int32_t nchunks;
  int32_t solve;             // read r from rbuf[st->acc] and run only in PH_NEED_GRAD
  const float* r;
  float* rbuf[kMaxTrials + 1];
  double* partials;          // per chunk
  SolverState* st;
};

struct AdjFinalArgs {
  const int32_t* col_chunk;  // nb + 1 chunk boundaries per column
  int32_t nb;
  int32_t solve;
  double scale;
  const double* partials;
  float* out;
  SolverState* st;
};

struct DecideArgs {
  const double* partials;    // [trial][nparts]
  int32_t nparts, nb;
  float* x;                  // x_k, overwritten by the accepted trial
  const float* g;
  SolverState* st;
  TraceDev* trace;
};

// ---- host-side objects ------------------------------------------------------------
struct Tuning {
  int fwd_grid_per_cu = 4;
  int adj_grid_per_cu = 8;
  int batch_iters = 32;        // iterations enqueued between host polls
};

}  // namespace imrt

struct imrt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int num_cu = 256;
  size_t max_lds = 65536;
  imrt::Tuning tune;
};

struct imrt_dose {
  imrt_ctx* ctx = nullptr;
  int32_t nv = 0, nb = 0;
  int64_t nnz = 0;
  // CSR (forward) and CSC (adjoint) copies of D
  int32_t* row_ptr = nullptr;
  int32_t* col_idx = nullptr;
  float* val = nullptr;
  int32_t* col_ptr = nullptr;
  int32_t* row_idx = nullptr;
  float* cval = nullptr;
  // forward row blocks and adjoint chunks
  int32_t nblocks = 0;
  int32_t* block_row = nullptr;
  int32_t nchunks = 0;
  int32_t* chunk_k = nullptr;
  int32_t* col_chunk = nullptr;
  // structure ids from the phantom builder (nullable)
  uint8_t* sid = nullptr;
  // scratch for plain products
  double* partials = nullptr;
  int32_t partials_len = 0;
};

struct imrt_plan {
  imrt_ctx* ctx = nullptr;
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
  float* xk = nullptr;
  float* gk = nullptr;
  float* vtmp = nullptr;          // nv scratch
  double* fwd_partials = nullptr; // kMaxTrials * fwd grid
  double* adj_partials = nullptr; // nchunks
  double* misc = nullptr;         // small reduction scratch
  imrt::SolverState* st = nullptr;
  imrt::TraceDev* trace = nullptr;
  int32_t trace_cap = 0;
  imrt::SolverState* st_host = nullptr;   // pinned, 2 slots
  double* misc_host = nullptr;            // pinned
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
int launch_forward(const imrt_ctx* ctx, const imrt_dose* D, const FwdArgs& a, int ntrials, int grid,
                   hipEvent_t before = nullptr, hipEvent_t after = nullptr);
int launch_adjoint(const imrt_ctx* ctx, const imrt_dose* D, const AdjArgs& a, const AdjFinalArgs& f,
                   hipEvent_t before = nullptr, hipEvent_t after = nullptr);
int launch_decide(const imrt_ctx* ctx, const DecideArgs& a, int ntrials);
int launch_sum(const imrt_ctx* ctx, const double* parts, int n, double* out);
int launch_project(const imrt_ctx* ctx, const float* x, const float* g, double lambda, int nb,
                   float* x_out, double* s_out);
int launch_normalize(const imrt_ctx* ctx, const float* w, int nb, float* v_out, double* norm_out);
int forward_grid(const imrt_ctx* ctx, const imrt_dose* D);
size_t forward_lds_bytes(int nb, int ntrials);

// phantom builder (build.hip)
int build_phantom(imrt_ctx* ctx, const imrt_geometry* g, imrt_dose* D);

// host preprocessing (api.hip)
int finish_dose(imrt_dose* D, const std::vector<int32_t>& row_ptr, const std::vector<int32_t>& col_ptr);

}  // namespace imrt
