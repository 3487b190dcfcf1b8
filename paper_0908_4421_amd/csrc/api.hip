// C ABI of libimrt: argument validation, device memory, host preprocessing of
// D (row blocks and adjoint chunks) and the stream-ordered solve driver.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "imrt_internal.h"

// Device memory of imrt_gradient_noalloc (residual, forward partials, adjoint
// pieces, objective total): one copy per device, held until the process
// ends.  Host code never passes this name to a kernel; it uses the address
// that hipGetSymbolAddress returned for the device (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[IMRT_NOALLOC_SCRATCH_BYTES];

namespace imrt {

namespace {
thread_local std::string g_err;

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  if (v == nullptr || *v == 0) return dflt;
  const int x = std::atoi(v);
  return x > 0 ? x : dflt;
}

template <typename T>
int dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * count);
  if (e == hipErrorOutOfMemory) return set_error(IMRT_ENOMEM, "hipMalloc: out of device memory");
  if (e != hipSuccess) return hip_error(e, "hipMalloc");
  return IMRT_OK;
}

template <typename T>
void dev_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

int use_device(const imrt_ctx* ctx) {
  IMRT_HIP(hipSetDevice(ctx->device));
  return IMRT_OK;
}

// Largest forward grid of either forward variant at the current settings.
int forward_grid_cap(imrt_ctx* ctx, const imrt_dose* D) {
  const int saved = ctx->tune.fwd_wave;
  int g = 1;
  for (int wave = 0; wave <= 1; ++wave)
    for (int nt : {1, 2}) {
      ctx->tune.fwd_wave = wave;
      g = std::max(g, forward_grid(ctx, D, nt));
    }
  ctx->tune.fwd_wave = saved;
  return g;
}

double pow2_at_least(double q) {
  int ex = 0;
  const double mant = std::frexp(q, &ex);
  return mant == 0.5 ? q : std::ldexp(1.0, ex);
}

}  // namespace

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_error(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return IMRT_EHIP;
}

// Device arrays of D: row and column pointers, and the four nonzero arrays,
// each followed by kPad zeroed entries so that 16-byte vector loads that
// straddle the end stay in bounds.
// Device address of `scratch` per device, looked up once per device with
// that device current (at context creation).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return set_error(IMRT_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return IMRT_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
  if (!p) return set_error(IMRT_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
  g_scratch_ptr[device] = p;
  return IMRT_OK;
}

unsigned char* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return static_cast<unsigned char*>(g_scratch_ptr[device]);
}

int alloc_nonzeros(imrt_dose* D) {
  const size_t nz = static_cast<size_t>(D->nnz) + kPad;
  const size_t nzc = csc_alloc(D->nnz);
  int rc;
  if ((rc = dev_alloc(&D->row_ptr, static_cast<size_t>(D->nv) + 1)) ||
      (rc = dev_alloc(&D->col_ptr, static_cast<size_t>(D->nb) + 1)) || (rc = dev_alloc(&D->col_idx, nz)) ||
      (rc = dev_alloc(&D->val, nz)) || (rc = dev_alloc(&D->row_idx, nzc)) || (rc = dev_alloc(&D->cval, nzc)))
    return rc;
  hipStream_t s = D->ctx->stream;
  const size_t off = static_cast<size_t>(D->nnz);
  IMRT_HIP(hipMemsetAsync(D->col_idx + off, 0, sizeof(int32_t) * kPad, s));
  IMRT_HIP(hipMemsetAsync(D->val + off, 0, sizeof(float) * kPad, s));
  // the CSC tile holding the last nonzero and everything after it start as zeros
  const size_t t0 = off & ~static_cast<size_t>(kTile - 1);
  IMRT_HIP(hipMemsetAsync(D->row_idx + t0, 0, sizeof(int32_t) * (nzc - t0), s));
  IMRT_HIP(hipMemsetAsync(D->cval + t0, 0, sizeof(float) * (nzc - t0), s));
  return IMRT_OK;
}

void partition_for_targets(int64_t nnz, int ta, int tf, int32_t* adj_min_nnz, int32_t* fwd_bpw) {
  nnz = std::max<int64_t>(nnz, 1);
  ta = std::max(ta, 1);
  tf = std::max(tf, 1);
  *adj_min_nnz = static_cast<int32_t>(std::min<int64_t>(32768, std::max<int64_t>(1024, (nnz + ta - 1) / ta)));
  const int64_t blocks = nnz / kWaveNnz + 1;
  *fwd_bpw = static_cast<int32_t>(
      std::min<int64_t>(4, std::max<int64_t>(1, blocks / (int64_t(forward_waves(1, 8)) * tf))));
}

void apply_partition_targets(const imrt_ctx* ctx, imrt_dose* D) {
  if (ctx->tune.part_adj_wgs > 0 && ctx->tune.part_fwd_wgs > 0) {
    partition_for_targets(D->nnz, ctx->tune.part_adj_wgs, ctx->tune.part_fwd_wgs, &D->adj_min_nnz, &D->fwd_bpw);
    D->fwd_waves = 8;
  }
}

// Row blocks for the forward pass (at most kFwdPartNnz nonzeros and
// kFwdRowsMax rows each, or one longer row alone), and the adjoint partition:
// workgroup w of G owns nonzeros [w*nnz/G, (w+1)*nnz/G) of the CSC arrays.
int finish_dose(imrt_dose* D, const std::vector<int32_t>& row_ptr, const std::vector<int32_t>& col_ptr) {
  if (D->fwd_st < 0)   // the forward layout, fixed with the first partition
    D->fwd_st = (D->storage == ST_F32 && D->nb <= 65536 && D->ctx->tune.fwd_col16) ? ST_F32C16 : D->storage;
  std::vector<int32_t> blocks, block_k0;
  blocks.push_back(0);
  int r = 0;
  while (r < D->nv) {
    const int start = r;
    int64_t nz = 0;
    while (r < D->nv && r - start < kFwdRowsMax) {
      const int64_t len = row_ptr[r + 1] - row_ptr[r];
      if (r > start && nz + len > kFwdPartNnz) break;
      nz += len;
      ++r;
      if (nz > kFwdPartNnz) break;
    }
    blocks.push_back(r);
  }
  for (int32_t b : blocks) block_k0.push_back(row_ptr[b]);
  // the same for one wave (at most wave_part_nnz nonzeros, which depends on
  // the storage, and kWaveRowsMax rows), except that a run of kGapRows or
  // more rows without nonzeros lies between blocks instead of inside one:
  // the wave forward never visits those rows (their penalty at zero dose is
  // a constant of the plan, and their residual is never gathered)
  const int wave_part = wave_part_nnz(D->fwd_st);
  const int nv = D->nv;
  std::vector<int32_t> run_end(static_cast<size_t>(nv) + 1);
  run_end[nv] = nv;
  for (int q = nv - 1; q >= 0; --q) run_end[q] = (row_ptr[q + 1] == row_ptr[q]) ? run_end[q + 1] : q;
  auto long_gap = [&](int q) { return run_end[q] - q >= kGapRows; };
  std::vector<std::pair<int32_t, int32_t>> wb;   // [first row, end row) of each block
  std::vector<std::pair<int32_t, int32_t>> gaps;
  r = 0;
  while (r < nv) {
    if (long_gap(r)) {
      gaps.emplace_back(r, run_end[r]);
      r = run_end[r];
      continue;
    }
    const int start = r;
    int64_t nz = 0;
    while (r < nv && r - start < kWaveRowsMax) {
      if (r > start && long_gap(r)) break;
      const int64_t len = row_ptr[r + 1] - row_ptr[r];
      if (r > start && nz + len > wave_part) break;
      nz += len;
      ++r;
      if (nz > wave_part) break;
    }
    wb.emplace_back(start, r);
  }
  if (wb.empty()) {
    // no nonzeros at all: one block of rows anyway (every pass has work)
    gaps.clear();
    wb.emplace_back(0, std::min(nv, kWaveRowsMax));
    for (int q = wb[0].second; q < nv; q += kWaveRowsMax) wb.emplace_back(q, std::min(nv, q + kWaveRowsMax));
  }
  // A wave's time is mostly a per-block latency, so every wave of the
  // default grid gets the same number of blocks: the blocks with the most
  // nonzeros are halved (by rows) until the count is a multiple of the waves.
  {
    const int nwb = static_cast<int>(wb.size());
    const int64_t waves =
        static_cast<int64_t>(wave_grid(D->ctx, nwb, 1, D->fwd_bpw, D->nb, D->fwd_st, D->fwd_waves)) *
        forward_waves(1, D->fwd_waves);
    const int64_t target = (nwb + waves - 1) / waves * waves;
    if (nwb > waves && target > nwb) {
      // max-heap of (nonzeros, block start row) over splittable blocks
      std::vector<std::pair<int64_t, int32_t>> heap;
      std::vector<int32_t> end_of(static_cast<size_t>(nv) + 1, -1);
      for (const auto& blk : wb) {
        end_of[blk.first] = blk.second;
        if (blk.second - blk.first > 1)
          heap.emplace_back(int64_t(row_ptr[blk.second]) - row_ptr[blk.first], blk.first);
      }
      std::make_heap(heap.begin(), heap.end());
      for (int64_t extra = target - nwb; extra > 0 && !heap.empty(); --extra) {
        std::pop_heap(heap.begin(), heap.end());
        const int32_t r0 = heap.back().second;
        heap.pop_back();
        const int32_t r1 = end_of[r0];
        const int64_t half = (int64_t(row_ptr[r0]) + row_ptr[r1]) / 2;
        int32_t m = r0 + 1;
        while (m < r1 - 1 && row_ptr[m] < half) ++m;
        end_of[r0] = m;
        end_of[m] = r1;
        wb.emplace_back(m, r1);
        if (m - r0 > 1) {
          heap.emplace_back(int64_t(row_ptr[m]) - row_ptr[r0], r0);
          std::push_heap(heap.begin(), heap.end());
        }
        if (r1 - m > 1) {
          heap.emplace_back(int64_t(row_ptr[r1]) - row_ptr[m], m);
          std::push_heap(heap.begin(), heap.end());
        }
      }
      for (auto& blk : wb) blk.second = end_of[blk.first];
      std::sort(wb.begin(), wb.end());
    }
  }
  std::vector<int32_t> wblocks, wblock_k0, wblock_end;
  for (const auto& blk : wb) {
    wblocks.push_back(blk.first);
    wblock_end.push_back(blk.second);
    wblock_k0.push_back(row_ptr[blk.first]);
  }
  wblocks.push_back(nv);
  wblock_k0.push_back(row_ptr[nv]);

  const int G = adjoint_grid_for(D->ctx, D->nnz, D->adj_min_nnz);
  const int64_t nnz = D->nnz;
  auto kw = [&](int64_t w) { return w * nnz / G; };
  std::vector<int32_t> wg_c0(G, 0), wg_c1(G, 0), col_wlo(D->nb), col_whi(D->nb);
  for (int w = 0; w < G; ++w) {
    wg_c0[w] = D->nb;
    wg_c1[w] = 0;
  }
  int w = 0;
  for (int c = 0; c < D->nb; ++c) {
    const int64_t cs = col_ptr[c], ce = col_ptr[c + 1];
    int lo, hi;
    if (ce == cs) {
      // empty column: the workgroup whose range holds its position (last one at the end)
      while (w + 1 < G && kw(w + 1) <= cs) ++w;
      lo = hi = w;
    } else {
      while (w + 1 < G && kw(w + 1) <= cs) ++w;
      lo = w;
      hi = w;
      while (hi + 1 < G && kw(hi + 1) < ce) ++hi;
    }
    col_wlo[c] = lo;
    col_whi[c] = hi;
    for (int v = lo; v <= hi; ++v) {
      wg_c0[v] = std::min(wg_c0[v], c);
      wg_c1[v] = std::max(wg_c1[v], c + 1);
    }
  }
  std::vector<int32_t> wg_cols(4 * static_cast<size_t>(G), 0);
  for (int v = 0; v < G; ++v) {
    if (wg_c1[v] == 0) continue;  // no columns
    const int c = wg_c0[v];
    wg_cols[4 * v] = c;
    wg_cols[4 * v + 1] = wg_c1[v];
    wg_cols[4 * v + 2] = static_cast<int32_t>(std::max<int64_t>(col_ptr[c], kw(v)));
    wg_cols[4 * v + 3] = static_cast<int32_t>(std::min<int64_t>(col_ptr[c + 1], kw(v + 1)));
  }
  D->nblocks = static_cast<int32_t>(blocks.size()) - 1;
  D->nwblocks = static_cast<int32_t>(wblocks.size()) - 1;
  D->gaps.swap(gaps);
  D->part_epoch += 1;
  D->adj_grid = G;
  // (a repartition replaces the previous tables)
  for (int32_t** p : {&D->block_row, &D->block_k0, &D->wblock_row, &D->wblock_k0, &D->wblock_end, &D->wg_cols,
                      &D->col_wlo, &D->col_whi})
    dev_free(*p);
  dev_free(D->col_kind);
  dev_free(D->pieces);
  dev_free(D->partials);
  int rc;
  if ((rc = dev_alloc(&D->block_row, blocks.size())) || (rc = dev_alloc(&D->block_k0, block_k0.size())) ||
      (rc = dev_alloc(&D->wblock_row, wblocks.size())) || (rc = dev_alloc(&D->wblock_k0, wblock_k0.size())) ||
      (rc = dev_alloc(&D->wblock_end, std::max<size_t>(wblock_end.size(), 1))) ||
      (rc = dev_alloc(&D->wg_cols, 4 * static_cast<size_t>(G))) ||
      (rc = dev_alloc(&D->col_wlo, static_cast<size_t>(D->nb))) ||
      (rc = dev_alloc(&D->col_whi, static_cast<size_t>(D->nb))) ||
      (rc = dev_alloc(&D->col_kind, static_cast<size_t>(D->nb))) ||
      (rc = dev_alloc(&D->pieces, 2 * static_cast<size_t>(G))))
    return rc;
  hipStream_t s = D->ctx->stream;
  IMRT_HIP(hipMemcpyAsync(D->block_row, blocks.data(), sizeof(int32_t) * blocks.size(), hipMemcpyHostToDevice, s));
  IMRT_HIP(hipMemcpyAsync(D->block_k0, block_k0.data(), sizeof(int32_t) * block_k0.size(), hipMemcpyHostToDevice, s));
  IMRT_HIP(hipMemcpyAsync(D->wblock_row, wblocks.data(), sizeof(int32_t) * wblocks.size(), hipMemcpyHostToDevice, s));
  IMRT_HIP(hipMemcpyAsync(D->wblock_k0, wblock_k0.data(), sizeof(int32_t) * wblock_k0.size(),
                          hipMemcpyHostToDevice, s));
  IMRT_HIP(hipMemcpyAsync(D->wblock_end, wblock_end.data(), sizeof(int32_t) * wblock_end.size(),
                          hipMemcpyHostToDevice, s));
  IMRT_HIP(hipMemcpyAsync(D->wg_cols, wg_cols.data(), sizeof(int32_t) * wg_cols.size(), hipMemcpyHostToDevice, s));
  IMRT_HIP(hipMemcpyAsync(D->col_wlo, col_wlo.data(), sizeof(int32_t) * D->nb, hipMemcpyHostToDevice, s));
  IMRT_HIP(hipMemcpyAsync(D->col_whi, col_whi.data(), sizeof(int32_t) * D->nb, hipMemcpyHostToDevice, s));
  std::vector<uint8_t> kind(D->nb);
  for (int c = 0; c < D->nb; ++c) kind[c] = static_cast<uint8_t>(std::min(col_whi[c] - col_wlo[c], 2));
  IMRT_HIP(hipMemcpyAsync(D->col_kind, kind.data(), D->nb, hipMemcpyHostToDevice, s));
  D->fwd_cap = forward_grid_cap(D->ctx, D);
  D->partials_len = kMaxTrials * (D->fwd_cap + 1) + 16;
  if ((rc = dev_alloc(&D->partials, D->partials_len))) return rc;
  IMRT_HIP(hipStreamSynchronize(s));
  return IMRT_OK;
}

}  // namespace imrt

using namespace imrt;

namespace {

void free_dose(imrt_dose* D) {
  if (!D) return;
  (void)hipSetDevice(D->device);
  dev_free(D->row_ptr);
  dev_free(D->col_idx);
  dev_free(D->val);
  dev_free(D->col_ptr);
  dev_free(D->row_idx);
  dev_free(D->cval);
  dev_free(D->col16);
  dev_free(D->val16);
  dev_free(D->cval16);
  dev_free(D->col_scale);
  dev_free(D->block_row);
  dev_free(D->block_k0);
  dev_free(D->wblock_row);
  dev_free(D->wblock_k0);
  dev_free(D->wblock_end);
  dev_free(D->wg_cols);
  dev_free(D->col_wlo);
  dev_free(D->col_whi);
  dev_free(D->col_kind);
  dev_free(D->vox);
  dev_free(D->vscratch);
  dev_free(D->pieces);
  dev_free(D->sid);
  dev_free(D->partials);
  delete D;
}

void free_plan(imrt_plan* P) {
  if (!P) return;
  (void)hipSetDevice(P->device);
  dev_free(P->sid);
  dev_free(P->table);
  dev_free(P->Tu_vox);
  dev_free(P->To_vox);
  for (auto& b : P->rbuf) dev_free(b);
  for (auto& b : P->xbuf) dev_free(b);
  dev_free(P->gk);
  dev_free(P->vtmp);
  dev_free(P->fwd_partials);
  dev_free(P->pieces);
  dev_free(P->pieces_col);
  dev_free(P->misc);
  dev_free(P->st);
  dev_free(P->trace);
  if (P->st_host) (void)hipHostFree(P->st_host);
  if (P->misc_host) (void)hipHostFree(P->misc_host);
  delete P;
}

int plan_ready(const imrt_plan* P) {
  if (!P) return set_error(IMRT_EINVAL, "plan is NULL");
  if (!P->have_struct) return set_error(IMRT_ENOTREADY, "structures not set (imrt_set_structures)");
  if (!P->have_pen) return set_error(IMRT_ENOTREADY, "penalties not set (imrt_set_penalties)");
  return IMRT_OK;
}

// A plan's partition-sized buffers follow its dose matrix's partition (which
// imrt_dose_repartition may change after the plan was created).
int plan_fit(imrt_plan* P) {
  const imrt_dose* D = P->dose;
  int rc = use_device(P->ctx);
  if (rc) return rc;
  const int cap = forward_grid_cap(P->ctx, D);
  if (cap > P->fwd_cap) {
    dev_free(P->fwd_partials);
    P->fwd_cap = 0;
    if ((rc = dev_alloc(&P->fwd_partials, static_cast<size_t>(kMaxTrials) * (cap + 1)))) return rc;
    P->fwd_cap = cap;
  }
  if (D->adj_grid > P->pieces_cap) {
    dev_free(P->pieces);
    P->pieces_cap = 0;
    if ((rc = dev_alloc(&P->pieces, 2 * static_cast<size_t>(D->adj_grid)))) return rc;
    P->pieces_cap = D->adj_grid;
  }
  return IMRT_OK;
}

int plan_use(imrt_plan* P) {
  const int rc = plan_ready(P);
  return rc ? rc : plan_fit(P);
}

// Objective of the voxels the wave forward skips (the runs of rows without
// nonzeros between its blocks): at zero dose each contributes
// F_j(0) = w_u min(-T_u, 0)^2 + w_o max(-T_o, 0)^2 (Eq. (1)), summed here in
// float64 in row order, once per set of structures, penalties, targets and
// partition.  The workgroup-wide forward visits every row: no constant then.
double plan_skip_objective(imrt_plan* P) {
  const imrt_dose* D = P->dose;
  if (P->ctx->tune.fwd_wave == 0) return 0.0;
  if (P->gskip_epoch == D->part_epoch) return P->G_skip;
  // skipped rows per structure (kept until the structures or the partition change)
  if (P->skip_hist_epoch != D->part_epoch) {
    P->skip_hist.assign(kMaxStruct, 0);
    for (const auto& gap : D->gaps)
      for (int32_t j = gap.first; j < gap.second; ++j) ++P->skip_hist[P->sid_host[j]];
    P->skip_hist_epoch = D->part_epoch;
  }
  auto F0 = [](double Tu, double To, double wu, double wo) {
    const double under = std::fmin(0.0 - Tu, 0.0);
    const double over = std::fmax(0.0 - To, 0.0);
    const double a = wu * under * under;
    const double b = wo * over * over;
    return a + b;
  };
  double G = 0.0;
  if (P->Tu_host.empty()) {
    for (int st = 0; st < P->nstruct; ++st)
      if (P->skip_hist[st] > 0) {
        const PenaltyDev& t = P->table_host[st];
        G += static_cast<double>(P->skip_hist[st]) * F0(t.T_u, t.T_o, t.w_u, t.w_o);
      }
  } else {
    for (const auto& gap : D->gaps)
      for (int32_t j = gap.first; j < gap.second; ++j) {
        const PenaltyDev& t = P->table_host[P->sid_host[j]];
        G += F0(static_cast<double>(P->Tu_host[j]), static_cast<double>(P->To_host[j]), t.w_u, t.w_o);
      }
  }
  P->G_skip = G;
  P->gskip_epoch = D->part_epoch;
  return G;
}

Penalties plan_penalties(const imrt_plan* P) {
  return Penalties{P->sid, P->table, P->Tu_vox, P->To_vox};
}

void set_plan_penalties(FwdArgs& a, const imrt_plan* P) {
  a.pen = plan_penalties(P);
  a.nstruct = P->nstruct;
}

// Bytes of the matrix streams one iteration reads: the forward layout's
// column index and value per nonzero, and the CSC's row index and value.
int64_t stream_bytes(const imrt_dose* D) {
  const int64_t fwd = (D->fwd_st == ST_F32) ? 8 : (D->fwd_st == ST_F32C16) ? 6 : 4;
  const int64_t adj = (D->storage == ST_F32) ? 8 : 6;
  return static_cast<int64_t>(D->nnz) * (fwd + adj);
}

// Cache policy of a solve pass's matrix streams (0 default, 2 non-temporal)
// under the context's stream_nt option.
int stream_policy(const imrt_ctx* ctx, int64_t bytes) {
  const int opt = ctx->tune.stream_nt;
  return (opt == 1 || (opt == 2 && bytes > kLlcBytes)) ? 2 : 0;
}

FwdArgs base_fwd(const imrt_dose* D) {
  FwdArgs a{};
  a.stream_cp = stream_policy(D->ctx, stream_bytes(D));
  a.row_ptr = D->row_ptr;
  a.col_idx = D->col_idx;
  a.val = D->val;
  a.col16 = D->col16;
  a.val16 = D->val16;
  a.col_scale = D->col_scale;
  a.storage = D->fwd_st;
  a.waves = D->fwd_waves;
  a.block_row = D->block_row;
  a.block_k0 = D->block_k0;
  a.nblocks = D->nblocks;
  a.wblock_row = D->wblock_row;
  a.wblock_k0 = D->wblock_k0;
  a.wblock_end = D->wblock_end;
  a.nwblocks = D->nwblocks;
  a.nv = D->nv;
  a.nb = D->nb;
  return a;
}

// Residual (nv) and iterate (nb) buffers 0..count-1.
int ensure_buffers(imrt_plan* P, int count) {
  for (int i = 0; i < count; ++i) {
    int rc;
    if (P->rbuf[i] == nullptr && (rc = dev_alloc(&P->rbuf[i], P->dose->nv))) return rc;
    if (P->xbuf[i] == nullptr && (rc = dev_alloc(&P->xbuf[i], P->dose->nb))) return rc;
  }
  return IMRT_OK;
}

// Objective (and optionally dose/residual) of x on the plan's stream; the
// float64 total lands in P->misc[slot].
int eval_forward(imrt_plan* P, const float* x, float* dose_out, float* r_out, int slot) {
  const imrt_dose* D = P->dose;
  FwdArgs a = base_fwd(D);
  a.mode = FWD_EVAL;
  set_plan_penalties(a, P);
  a.x = x;
  a.d_out = dose_out;
  a.r_out = r_out;
  a.partials = P->fwd_partials;
  const int grid = std::min(forward_grid(P->ctx, D), P->fwd_cap);
  int rc = launch_forward(P->ctx, D, a, 1, grid);
  if (rc) return rc;
  return launch_sum(P->ctx, P->fwd_partials, grid, P->misc + slot, plan_skip_objective(P));
}

AdjArgs base_adj(const imrt_dose* D) {
  AdjArgs a{};
  a.stream_cp = stream_policy(D->ctx, stream_bytes(D));
  a.row_idx = D->row_idx;
  a.val = D->cval;
  a.val16 = D->cval16;
  a.col_scale = D->col_scale;
  a.storage = D->storage;
  a.col_ptr = D->col_ptr;
  a.wg_cols = D->wg_cols;
  a.col_wlo = D->col_wlo;
  a.col_whi = D->col_whi;
  a.col_kind = D->col_kind;
  a.nnz = D->nnz;
  a.nv = D->nv;
  a.nb = D->nb;
  a.grid = D->adj_grid;
  a.xcd_map = D->ctx->tune.adj_xcd;
  return a;
}

// y = scale * D^T r with the dose's own piece scratch.
int adjoint_into(const imrt_ctx* ctx, const imrt_dose* D, const float* r, double scale, float* out) {
  AdjArgs a = base_adj(D);
  a.solve = 0;
  a.r = r;
  a.pieces = D->pieces;
  a.out = out;
  a.scale = scale;
  return launch_adjoint(ctx, D, a, 1);
}

int fetch_misc(imrt_plan* P, int n) {
  IMRT_HIP(hipMemcpyAsync(P->misc_host, P->misc, sizeof(double) * n, hipMemcpyDeviceToHost, P->ctx->stream));
  IMRT_HIP(hipStreamSynchronize(P->ctx->stream));
  return IMRT_OK;
}

}  // namespace

extern "C" {

const char* imrt_last_error(void) { return imrt::g_err.c_str(); }

int imrt_ctx_create(int device, void* hip_stream, imrt_ctx** out) {
  if (!out) return set_error(IMRT_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  IMRT_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_error(IMRT_EINVAL, "device index out of range");
  IMRT_HIP(hipSetDevice(device));
  int rc0 = noalloc_scratch_init(device);
  if (rc0) return rc0;
  auto* c = new (std::nothrow) imrt_ctx();
  if (!c) return set_error(IMRT_ENOMEM, "host allocation failed");
  c->device = device;
  int ncu = 0, lds = 0, culds = 0;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
  (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  (void)hipDeviceGetAttribute(&culds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device);
  if (ncu > 0) c->num_cu = ncu;
  if (lds > 0) c->max_lds = static_cast<size_t>(lds);
  c->cu_lds = std::max(c->max_lds, culds > 0 ? static_cast<size_t>(culds) : c->max_lds);
  c->tune.fwd_grid_per_cu = std::min(64, env_int("IMRT_FWD_WG_PER_CU", c->tune.fwd_grid_per_cu));
  c->tune.adj_grid_per_cu = std::min(64, env_int("IMRT_ADJ_WG_PER_CU", c->tune.adj_grid_per_cu));
  c->tune.batch_iters = env_int("IMRT_BATCH_ITERS", c->tune.batch_iters);
  c->tune.adj_min_nnz = env_int("IMRT_ADJ_MIN_NNZ", c->tune.adj_min_nnz);
  c->tune.fwd_bpw = std::min(1024, env_int("IMRT_FWD_BLOCKS_PER_WAVE", c->tune.fwd_bpw));
  if (const char* f = std::getenv("IMRT_FWD_WAVE")) c->tune.fwd_wave = (std::atoi(f) != 0) ? 1 : 0;
  if (const char* f = std::getenv("IMRT_ADJ_XCD")) c->tune.adj_xcd = (std::atoi(f) != 0) ? 1 : 0;
  if (const char* f = std::getenv("IMRT_VOXEL_TILES")) c->tune.voxel_tiles = (std::atoi(f) != 0) ? 1 : 0;
  if (const char* f = std::getenv("IMRT_FWD_COL16")) c->tune.fwd_col16 = (std::atoi(f) != 0) ? 1 : 0;
  c->stream = static_cast<hipStream_t>(hip_stream);  // NULL: the device's null stream
  *out = c;
  return IMRT_OK;
}

int imrt_ctx_destroy(imrt_ctx* ctx) {
  if (!ctx) return IMRT_OK;
  (void)hipSetDevice(ctx->device);
  delete ctx;
  return IMRT_OK;
}

int imrt_ctx_stream(const imrt_ctx* ctx, void** hip_stream_out) {
  if (!ctx || !hip_stream_out) return set_error(IMRT_EINVAL, "ctx or out is NULL");
  *hip_stream_out = ctx->stream;
  return IMRT_OK;
}

namespace {
int* option_slot(imrt_ctx* ctx, const char* name, int64_t* lo) {
  if (!name) return nullptr;
  const std::string n(name);
  *lo = 1;
  if (n == "fwd_wg_per_cu") return &ctx->tune.fwd_grid_per_cu;
  if (n == "adj_wg_per_cu") return &ctx->tune.adj_grid_per_cu;
  if (n == "batch_iters") return &ctx->tune.batch_iters;
  if (n == "adj_min_nnz") {
    *lo = 16;
    return &ctx->tune.adj_min_nnz;
  }
  if (n == "fwd_wave") {
    *lo = 0;
    return &ctx->tune.fwd_wave;
  }
  if (n == "fwd_blocks_per_wave") return &ctx->tune.fwd_bpw;
  if (n == "fwd_col16") {
    *lo = 0;
    return &ctx->tune.fwd_col16;
  }
  if (n == "serve_adjoint_workgroups") return &ctx->tune.serve_adj_wgs;
  if (n == "serve_forward_workgroups") return &ctx->tune.serve_fwd_wgs;
  if (n == "serve_groups_per_poll") return &ctx->tune.serve_groups;
  if (n == "serve_shared_adjoint") {
    *lo = 0;
    return &ctx->tune.serve_shared_adj;
  }
  if (n == "adj_xcd") {
    *lo = 0;
    return &ctx->tune.adj_xcd;
  }
  if (n == "voxel_tiles") {
    *lo = 0;
    return &ctx->tune.voxel_tiles;
  }
  if (n == "stream_nt") {
    *lo = 0;
    return &ctx->tune.stream_nt;
  }
  return nullptr;
}
}  // namespace

int imrt_ctx_set_option(imrt_ctx* ctx, const char* name, int64_t value) {
  if (!ctx) return set_error(IMRT_EINVAL, "ctx is NULL");
  int64_t lo = 0;
  int* slot = option_slot(ctx, name, &lo);
  if (!slot) return set_error(IMRT_EINVAL, std::string("unknown option: ") + (name ? name : "(null)"));
  const std::string nm(name);
  const int64_t hi = (nm == "fwd_wave" || nm == "adj_xcd" || nm == "voxel_tiles" || nm == "fwd_col16" ||
                      nm == "serve_shared_adjoint")
                         ? 1
                     : (nm == "fwd_wg_per_cu" || nm == "adj_wg_per_cu")         ? 64
                     : (nm == "fwd_blocks_per_wave")                                         ? 1024
                     : (nm == "serve_adjoint_workgroups" || nm == "serve_forward_workgroups") ? 65536
                     : (nm == "serve_groups_per_poll")                                      ? 4096
                     : (nm == "stream_nt")                                                  ? 2
                                                                                 : (int64_t(1) << 30);
  if (value < lo || value > hi) return set_error(IMRT_EINVAL, std::string("value out of range for ") + name);
  *slot = static_cast<int>(value);
  return IMRT_OK;
}

int imrt_ctx_get_option(const imrt_ctx* ctx, const char* name, int64_t* value) {
  if (!ctx || !value) return set_error(IMRT_EINVAL, "ctx or value is NULL");
  int64_t lo = 0;
  int* slot = option_slot(const_cast<imrt_ctx*>(ctx), name, &lo);
  if (!slot) return set_error(IMRT_EINVAL, std::string("unknown option: ") + (name ? name : "(null)"));
  *value = *slot;
  return IMRT_OK;
}

int imrt_build_dose_matrix(imrt_ctx* ctx, const imrt_geometry* geom, imrt_dtype storage, imrt_dose** out,
                           uint8_t* voxel_struct_out) {
  if (!ctx || !geom || !out) return set_error(IMRT_EINVAL, "ctx, geom or out is NULL");
  *out = nullptr;
  if (storage != IMRT_F32 && storage != IMRT_BF16 && storage != IMRT_F16)
    return set_error(IMRT_EINVAL, "storage must be IMRT_F32, IMRT_BF16 or IMRT_F16");
  int rc = use_device(ctx);
  if (rc) return rc;
  auto* D = new (std::nothrow) imrt_dose();
  if (!D) return set_error(IMRT_ENOMEM, "host allocation failed");
  D->ctx = ctx;
  D->device = ctx->device;
  D->storage = storage;   // the row-block partition depends on it
  D->adj_min_nnz = ctx->tune.adj_min_nnz;
  D->fwd_bpw = ctx->tune.fwd_bpw;
  try {
    rc = build_phantom(ctx, geom, D);
    if (rc == IMRT_OK) rc = store16(D, storage);
  } catch (const std::bad_alloc&) {
    rc = set_error(IMRT_ENOMEM, "host allocation failed");
  }
  if (rc == IMRT_OK && D->vox) {
    const hipError_t e = hipMalloc(reinterpret_cast<void**>(&D->vscratch), sizeof(float) * D->nv);
    if (e != hipSuccess) rc = hip_error(e, "hipMalloc(permutation scratch)");
  }
  if (rc == IMRT_OK && voxel_struct_out) {
    std::vector<uint8_t> ids(D->nv);
    const hipError_t e = hipMemcpy(ids.data(), D->sid, D->nv, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_error(e, "hipMemcpy(voxel_struct)");
    for (int32_t p = 0; rc == IMRT_OK && p < D->nv; ++p) voxel_struct_out[D->vox ? D->vox_host[p] : p] = ids[p];
  }
  if (rc) {
    free_dose(D);
    return rc;
  }
  *out = D;
  return IMRT_OK;
}

int imrt_dose_from_csr(imrt_ctx* ctx, int32_t nv, int32_t nb, int64_t nnz, const int32_t* row_ptr,
                       const int32_t* col_idx, const float* val, imrt_dtype storage, imrt_dose** out) {
  if (!ctx || !out || !row_ptr) return set_error(IMRT_EINVAL, "ctx, out or row_ptr is NULL");
  *out = nullptr;
  if (storage != IMRT_F32 && storage != IMRT_BF16 && storage != IMRT_F16)
    return set_error(IMRT_EINVAL, "storage must be IMRT_F32, IMRT_BF16 or IMRT_F16");
  if (storage != IMRT_F32 && nb > 65536)
    return set_error(IMRT_EUNSUPPORTED, "16-bit storage needs nb <= 65536 (16-bit column indices)");
  if (nv <= 0 || nb <= 0) return set_error(IMRT_EINVAL, "nv and nb must be positive");
  if (nnz < 0 || nnz >= (int64_t(1) << 31)) return set_error(IMRT_EINVAL, "nnz must be in [0, 2^31)");
  if (nnz > 0 && (!col_idx || !val)) return set_error(IMRT_EINVAL, "col_idx or val is NULL");
  if (row_ptr[0] != 0 || row_ptr[nv] != nnz) return set_error(IMRT_EINVAL, "row_ptr must start at 0 and end at nnz");
  for (int32_t j = 0; j < nv; ++j) {
    if (row_ptr[j + 1] < row_ptr[j]) return set_error(IMRT_EINVAL, "row_ptr is decreasing");
    for (int32_t k = row_ptr[j]; k < row_ptr[j + 1]; ++k) {
      if (col_idx[k] < 0 || col_idx[k] >= nb) return set_error(IMRT_EINVAL, "column index out of range");
      if (k > row_ptr[j] && col_idx[k] <= col_idx[k - 1])
        return set_error(IMRT_EINVAL, "column indices must increase strictly within a row");
      if (!(val[k] >= 0.0f) || !std::isfinite(val[k])) return set_error(IMRT_EINVAL, "values must be finite and >= 0");
    }
  }
  int rc = use_device(ctx);
  if (rc) return rc;
  auto* D = new (std::nothrow) imrt_dose();
  if (!D) return set_error(IMRT_ENOMEM, "host allocation failed");
  D->ctx = ctx;
  D->device = ctx->device;
  D->nv = nv;
  D->nb = nb;
  D->nnz = nnz;
  D->storage = storage;   // the row-block partition depends on it
  D->adj_min_nnz = ctx->tune.adj_min_nnz;
  D->fwd_bpw = ctx->tune.fwd_bpw;
  try {
    // CSC by a stable counting sort over columns: rows stay ascending.
    std::vector<int32_t> rp(row_ptr, row_ptr + nv + 1), cp(nb + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) cp[col_idx[k] + 1]++;
    for (int i = 0; i < nb; ++i) cp[i + 1] += cp[i];
    // (stored in the tiled slot order of the CSC arrays; unused slots zero)
    const size_t nzc = csc_alloc(nnz);
    std::vector<int32_t> ri(nzc, 0), fill(cp.begin(), cp.end() - 1);
    std::vector<float> cv(nzc, 0.0f);
    for (int32_t j = 0; j < nv; ++j)
      for (int32_t k = row_ptr[j]; k < row_ptr[j + 1]; ++k) {
        const int64_t p = csc_slot(fill[col_idx[k]]++);
        ri[p] = j;
        cv[p] = val[k];
      }
    hipStream_t s = ctx->stream;
    if ((rc = alloc_nonzeros(D))) {
      free_dose(D);
      return rc;
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(D->row_ptr, row_ptr, sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && nnz) e = hipMemcpyAsync(D->col_idx, col_idx, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && nnz) e = hipMemcpyAsync(D->val, val, sizeof(float) * nnz, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(D->col_ptr, cp.data(), sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(D->row_idx, ri.data(), sizeof(int32_t) * nzc, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(D->cval, cv.data(), sizeof(float) * nzc, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      free_dose(D);
      return hip_error(e, "upload of D");
    }
    apply_partition_targets(ctx, D);
    rc = finish_dose(D, rp, cp);
    if (rc == IMRT_OK) rc = store16(D, storage);
  } catch (const std::bad_alloc&) {
    rc = set_error(IMRT_ENOMEM, "host allocation failed");
  }
  if (rc) {
    free_dose(D);
    return rc;
  }
  *out = D;
  return IMRT_OK;
}

int imrt_dose_info(const imrt_dose* dose, int32_t* nv, int32_t* nb, int64_t* nnz) {
  if (!dose) return set_error(IMRT_EINVAL, "dose is NULL");
  if (nv) *nv = dose->nv;
  if (nb) *nb = dose->nb;
  if (nnz) *nnz = dose->nnz;
  return IMRT_OK;
}

namespace {

// float64 value of a 16-bit code (bfloat16 or binary16 bit pattern).
double code_value_host(uint16_t h, int storage) {
  if (storage == ST_BF16) {
    const uint32_t b = static_cast<uint32_t>(h) << 16;
    float f;
    std::memcpy(&f, &b, sizeof f);
    return f;
  }
  const int e = (h >> 10) & 31, m = h & 1023;
  const double v = (e == 0) ? std::ldexp(static_cast<double>(m), -24) : std::ldexp(static_cast<double>(m + 1024), e - 25);
  return (h & 0x8000) ? -v : v;
}

// Host copies of D in the caller's voxel order: float32 values (for 16-bit
// storage the float32 rounding of s_i q_ij) and, for 16-bit storage, the
// codes themselves.
int export_dose(const imrt_dose* D, int32_t* row_ptr, int32_t* col_idx, float* val, int32_t* col_ptr,
                int32_t* row_idx, float* cval, uint8_t* voxel_struct, uint16_t* val_code, uint16_t* cval_code,
                float* col_scale) {
  int rc = use_device(D->ctx);
  if (rc) return rc;
  if (voxel_struct && !D->sid) return set_error(IMRT_EINVAL, "this dose matrix has no structure ids");
  const bool s16 = D->storage != ST_F32;
  if ((val_code || cval_code || col_scale) && !s16)
    return set_error(IMRT_EINVAL, "this dose matrix stores float32 values, not 16-bit codes");
  hipStream_t s = D->ctx->stream;
  const int nv = D->nv, nb = D->nb;
  const size_t nz = static_cast<size_t>(D->nnz);
  const bool perm = D->vox != nullptr;
  try {
    // internal arrays (CSC back in plain column-major order), then the
    // caller's voxel order: rows of D and row indices of the CSC mapped by vox
    const bool want_csr = row_ptr || col_idx || val || val_code;
    const bool want_csc = row_idx || cval || cval_code;
    std::vector<int32_t> rp(want_csr ? nv + 1 : 0), ci(want_csr ? nz : 0), cp(nb + 1), ri;
    std::vector<float> va(want_csr ? nz : 0), cv, sc(s16 ? nb : 0);
    std::vector<uint16_t> qa(want_csr && s16 ? nz : 0), qc, c16(want_csr && s16 ? nz : 0);
    std::vector<uint8_t> sid(voxel_struct ? nv : 0);
    if (s16) IMRT_HIP(hipMemcpyAsync(sc.data(), D->col_scale, sizeof(float) * nb, hipMemcpyDeviceToHost, s));
    if (want_csr) {
      IMRT_HIP(hipMemcpyAsync(rp.data(), D->row_ptr, sizeof(int32_t) * (nv + 1), hipMemcpyDeviceToHost, s));
      if (nz && !s16) {
        IMRT_HIP(hipMemcpyAsync(ci.data(), D->col_idx, sizeof(int32_t) * nz, hipMemcpyDeviceToHost, s));
        IMRT_HIP(hipMemcpyAsync(va.data(), D->val, sizeof(float) * nz, hipMemcpyDeviceToHost, s));
      } else if (nz) {
        IMRT_HIP(hipMemcpyAsync(c16.data(), D->col16, sizeof(uint16_t) * nz, hipMemcpyDeviceToHost, s));
        IMRT_HIP(hipMemcpyAsync(qa.data(), D->val16, sizeof(uint16_t) * nz, hipMemcpyDeviceToHost, s));
      }
    }
    IMRT_HIP(hipMemcpyAsync(cp.data(), D->col_ptr, sizeof(int32_t) * (nb + 1), hipMemcpyDeviceToHost, s));
    IMRT_HIP(hipStreamSynchronize(s));
    if (want_csr && s16)
      for (size_t k = 0; k < nz; ++k) {
        ci[k] = c16[k];
        va[k] = static_cast<float>(static_cast<double>(sc[ci[k]]) * code_value_host(qa[k], D->storage));
      }
    if (want_csc && nz) {
      const size_t nzc = csc_alloc(D->nnz);
      std::vector<int32_t> rit(nzc);
      std::vector<float> cvt(s16 ? 0 : nzc);
      std::vector<uint16_t> qct(s16 ? nzc : 0);
      IMRT_HIP(hipMemcpyAsync(rit.data(), D->row_idx, sizeof(int32_t) * nzc, hipMemcpyDeviceToHost, s));
      if (s16) IMRT_HIP(hipMemcpyAsync(qct.data(), D->cval16, sizeof(uint16_t) * nzc, hipMemcpyDeviceToHost, s));
      else IMRT_HIP(hipMemcpyAsync(cvt.data(), D->cval, sizeof(float) * nzc, hipMemcpyDeviceToHost, s));
      IMRT_HIP(hipStreamSynchronize(s));
      ri.resize(nz);
      cv.resize(nz);
      if (s16) qc.resize(nz);
      for (int32_t c = 0; c < nb; ++c)
        for (int32_t k = cp[c]; k < cp[c + 1]; ++k) {
          const int64_t p = csc_slot(k);
          ri[k] = rit[p];
          if (s16) {
            qc[k] = qct[p];
            cv[k] = static_cast<float>(static_cast<double>(sc[c]) * code_value_host(qct[p], D->storage));
          } else {
            cv[k] = cvt[p];
          }
        }
    }
    if (voxel_struct) IMRT_HIP(hipMemcpyAsync(sid.data(), D->sid, nv, hipMemcpyDeviceToHost, s));
    IMRT_HIP(hipStreamSynchronize(s));
    if (col_ptr) std::memcpy(col_ptr, cp.data(), sizeof(int32_t) * (nb + 1));
    if (col_scale && nb) std::memcpy(col_scale, sc.data(), sizeof(float) * nb);
    if (!perm) {
      if (row_ptr) std::memcpy(row_ptr, rp.data(), sizeof(int32_t) * (nv + 1));
      if (col_idx && nz) std::memcpy(col_idx, ci.data(), sizeof(int32_t) * nz);
      if (val && nz) std::memcpy(val, va.data(), sizeof(float) * nz);
      if (val_code && nz) std::memcpy(val_code, qa.data(), sizeof(uint16_t) * nz);
      if (row_idx && nz) std::memcpy(row_idx, ri.data(), sizeof(int32_t) * nz);
      if (cval && nz) std::memcpy(cval, cv.data(), sizeof(float) * nz);
      if (cval_code && nz) std::memcpy(cval_code, qc.data(), sizeof(uint16_t) * nz);
      if (voxel_struct) std::memcpy(voxel_struct, sid.data(), nv);
      return IMRT_OK;
    }
    const std::vector<int32_t>& vox = D->vox_host;
    std::vector<int32_t> ipos(nv);
    for (int32_t p = 0; p < nv; ++p) ipos[vox[p]] = p;
    if (want_csr) {
      int64_t k = 0;
      for (int32_t jv = 0; jv < nv; ++jv) {
        const int32_t p = ipos[jv];
        if (row_ptr) row_ptr[jv] = static_cast<int32_t>(k);
        for (int32_t e = rp[p]; e < rp[p + 1]; ++e, ++k) {
          if (col_idx) col_idx[k] = ci[e];
          if (val) val[k] = va[e];
          if (val_code) val_code[k] = qa[e];
        }
      }
      if (row_ptr) row_ptr[nv] = static_cast<int32_t>(k);
    }
    if (want_csc) {
      std::vector<int32_t> order;
      for (int32_t c = 0; c < nb; ++c) {
        order.clear();
        for (int32_t e = cp[c]; e < cp[c + 1]; ++e) order.push_back(e);
        std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return vox[ri[x]] < vox[ri[y]]; });
        for (int32_t e = cp[c]; e < cp[c + 1]; ++e) {
          const int32_t f = order[e - cp[c]];
          if (row_idx) row_idx[e] = vox[ri[f]];
          if (cval) cval[e] = cv[f];
          if (cval_code) cval_code[e] = qc[f];
        }
      }
    }
    if (voxel_struct)
      for (int32_t p = 0; p < nv; ++p) voxel_struct[vox[p]] = sid[p];
  } catch (const std::bad_alloc&) {
    return set_error(IMRT_ENOMEM, "host allocation failed");
  }
  return IMRT_OK;
}

}  // namespace

int imrt_dose_export(const imrt_dose* D, int32_t* row_ptr, int32_t* col_idx, float* val, int32_t* col_ptr,
                     int32_t* row_idx, float* cval, uint8_t* voxel_struct) {
  if (!D) return set_error(IMRT_EINVAL, "dose is NULL");
  return export_dose(D, row_ptr, col_idx, val, col_ptr, row_idx, cval, voxel_struct, nullptr, nullptr, nullptr);
}

int imrt_dose_export_codes(const imrt_dose* D, uint16_t* val_code, uint16_t* cval_code, float* col_scale) {
  if (!D) return set_error(IMRT_EINVAL, "dose is NULL");
  return export_dose(D, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, val_code, cval_code, col_scale);
}

int imrt_dose_storage(const imrt_dose* D, int32_t* storage) {
  if (!D || !storage) return set_error(IMRT_EINVAL, "dose or storage is NULL");
  *storage = D->storage;
  return IMRT_OK;
}

int imrt_dose_apply(const imrt_dose* D, const float* x_dev, float* d_dev) {
  if (!D || !x_dev || !d_dev) return set_error(IMRT_EINVAL, "dose, x or d is NULL");
  int rc = use_device(D->ctx);
  if (rc) return rc;
  FwdArgs a = base_fwd(D);
  a.mode = FWD_PLAIN;
  a.x = x_dev;
  a.d_out = D->vox ? D->vscratch : d_dev;
  a.partials = D->partials;
  // rows the wave blocks skip have no nonzeros: their dose is 0
  if (!D->gaps.empty() && D->ctx->tune.fwd_wave && (rc = launch_zero(D->ctx, a.d_out, D->nv))) return rc;
  if ((rc = launch_forward(D->ctx, D, a, 1, std::min(forward_grid(D->ctx, D), D->fwd_cap)))) return rc;
  return D->vox ? launch_permute(D->ctx, D->vscratch, D->vox, D->nv, d_dev, true) : IMRT_OK;
}

int imrt_dose_apply_transpose(const imrt_dose* D, const float* r_dev, float* y_dev) {
  if (!D || !r_dev || !y_dev) return set_error(IMRT_EINVAL, "dose, r or y is NULL");
  int rc = use_device(D->ctx);
  if (rc) return rc;
  if (D->vox) {
    if ((rc = launch_permute(D->ctx, r_dev, D->vox, D->nv, D->vscratch, false))) return rc;
    r_dev = D->vscratch;
  }
  return adjoint_into(D->ctx, D, r_dev, 1.0, y_dev);
}

int imrt_dose_destroy(imrt_dose* dose) {
  free_dose(dose);
  return IMRT_OK;
}

int imrt_plan_create(imrt_ctx* ctx, const imrt_dose* dose, imrt_plan** out) {
  if (!ctx || !dose || !out) return set_error(IMRT_EINVAL, "ctx, dose or out is NULL");
  *out = nullptr;
  if (dose->ctx->device != ctx->device) return set_error(IMRT_EINVAL, "dose lives on another device");
  int rc = use_device(ctx);
  if (rc) return rc;
  auto* P = new (std::nothrow) imrt_plan();
  if (!P) return set_error(IMRT_ENOMEM, "host allocation failed");
  P->ctx = ctx;
  P->device = ctx->device;
  P->dose = dose;
  const int grid = forward_grid_cap(ctx, dose);
  P->fwd_cap = grid;
  P->pieces_cap = dose->adj_grid;
  if ((rc = dev_alloc(&P->sid, dose->nv)) || (rc = dev_alloc(&P->table, kMaxStruct)) ||
      (rc = ensure_buffers(P, 2)) || (rc = dev_alloc(&P->gk, dose->nb)) || (rc = dev_alloc(&P->vtmp, dose->nv)) ||
      (rc = dev_alloc(&P->fwd_partials, static_cast<size_t>(kMaxTrials) * (grid + 1))) ||
      (rc = dev_alloc(&P->pieces, 2 * static_cast<size_t>(dose->adj_grid))) ||
      (rc = dev_alloc(&P->pieces_col, 2 * static_cast<size_t>(dose->nb))) || (rc = dev_alloc(&P->misc, 16)) ||
      (rc = dev_alloc(&P->st, 2))) {
    free_plan(P);
    return rc;
  }
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&P->st_host), sizeof(SolverState) * 2);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&P->misc_host), sizeof(double) * 16);
  if (e != hipSuccess) {
    free_plan(P);
    return hip_error(e, "hipHostMalloc");
  }
  *out = P;
  return IMRT_OK;
}

int imrt_set_structures(imrt_plan* P, const uint8_t* voxel_struct, int32_t nstruct) {
  if (!P) return set_error(IMRT_EINVAL, "plan is NULL");
  if (nstruct <= 0 || nstruct > kMaxStruct) return set_error(IMRT_EINVAL, "nstruct must be in [1, 256]");
  int rc = use_device(P->ctx);
  if (rc) return rc;
  const imrt_dose* D = P->dose;
  std::vector<uint8_t> ids;
  try {
    ids.resize(D->nv);
  } catch (const std::bad_alloc&) {
    return set_error(IMRT_ENOMEM, "host allocation failed");
  }
  if (voxel_struct) {
    // caller's voxel order to the internal one
    for (int32_t p = 0; p < D->nv; ++p) ids[p] = voxel_struct[D->vox ? D->vox_host[p] : p];
  } else {
    if (!D->sid) return set_error(IMRT_EINVAL, "NULL structure ids need a dose matrix from imrt_build_dose_matrix");
    IMRT_HIP(hipMemcpy(ids.data(), D->sid, D->nv, hipMemcpyDeviceToHost));
  }
  std::vector<char> present(kMaxStruct, 0);
  for (int32_t j = 0; j < D->nv; ++j) {
    if (ids[j] >= nstruct) return set_error(IMRT_EINVAL, "structure id >= nstruct");
    present[ids[j]] = 1;
  }
  IMRT_HIP(hipMemcpy(P->sid, ids.data(), D->nv, hipMemcpyHostToDevice));
  P->sid_host.swap(ids);
  P->gskip_epoch = -1;
  P->skip_hist_epoch = -1;
  P->nstruct = nstruct;
  P->have_struct = true;
  P->have_pen = false;  // the table must match the new structure count
  return IMRT_OK;
}

int imrt_set_penalties(imrt_plan* P, const imrt_penalty* table) {
  if (!P || !table) return set_error(IMRT_EINVAL, "plan or table is NULL");
  if (!P->have_struct) return set_error(IMRT_ENOTREADY, "set structures before penalties");
  int rc = use_device(P->ctx);
  if (rc) return rc;
  std::vector<PenaltyDev> t(P->nstruct);
  for (int s = 0; s < P->nstruct; ++s) {
    const imrt_penalty& p = table[s];
    if (!std::isfinite(p.T_under) || !std::isfinite(p.T_over) || !std::isfinite(p.w_under) ||
        !std::isfinite(p.w_over))
      return set_error(IMRT_EINVAL, "penalty parameters must be finite");
    if (p.w_under < 0 || p.w_over < 0) return set_error(IMRT_EINVAL, "penalty weights must be >= 0");
    t[s] = PenaltyDev{p.T_under, p.T_over, p.w_under, p.w_over};
  }
  // largest weight over the structures that occur among the voxels
  std::vector<uint8_t> ids(P->dose->nv);
  IMRT_HIP(hipMemcpy(ids.data(), P->sid, P->dose->nv, hipMemcpyDeviceToHost));
  std::vector<char> present(kMaxStruct, 0);
  for (uint8_t s : ids) present[s] = 1;
  double wmax = 0.0;
  for (int s = 0; s < P->nstruct; ++s)
    if (present[s]) wmax = std::max(wmax, std::max(t[s].w_u, t[s].w_o));
  IMRT_HIP(hipMemcpy(P->table, t.data(), sizeof(PenaltyDev) * P->nstruct, hipMemcpyHostToDevice));
  P->table_host.swap(t);
  P->gskip_epoch = -1;
  P->w_max = wmax;
  P->have_pen = true;
  return IMRT_OK;
}

int imrt_set_voxel_targets(imrt_plan* P, const float* T_under, const float* T_over) {
  if (!P) return set_error(IMRT_EINVAL, "plan is NULL");
  int rc = use_device(P->ctx);
  if (rc) return rc;
  if (!T_under && !T_over) {
    dev_free(P->Tu_vox);
    dev_free(P->To_vox);
    P->Tu_host.clear();
    P->To_host.clear();
    P->gskip_epoch = -1;
    return IMRT_OK;
  }
  if (!T_under || !T_over) return set_error(IMRT_EINVAL, "give both T_under and T_over, or neither");
  const int nv = P->dose->nv;
  for (int j = 0; j < nv; ++j)
    if (!std::isfinite(T_under[j]) || !std::isfinite(T_over[j]))
      return set_error(IMRT_EINVAL, "voxel targets must be finite");
  if (!P->Tu_vox && (rc = dev_alloc(&P->Tu_vox, nv))) return rc;
  if (!P->To_vox && (rc = dev_alloc(&P->To_vox, nv))) return rc;
  const imrt_dose* D = P->dose;
  std::vector<float> tu, to;
  if (D->vox) {
    tu.resize(nv);
    to.resize(nv);
    for (int32_t p = 0; p < nv; ++p) {
      tu[p] = T_under[D->vox_host[p]];
      to[p] = T_over[D->vox_host[p]];
    }
    T_under = tu.data();
    T_over = to.data();
  }
  IMRT_HIP(hipMemcpy(P->Tu_vox, T_under, sizeof(float) * nv, hipMemcpyHostToDevice));
  IMRT_HIP(hipMemcpy(P->To_vox, T_over, sizeof(float) * nv, hipMemcpyHostToDevice));
  P->Tu_host.assign(T_under, T_under + nv);
  P->To_host.assign(T_over, T_over + nv);
  P->gskip_epoch = -1;
  return IMRT_OK;
}

int imrt_evaluate_objective(imrt_plan* P, const float* x_dev, double* G_out, float* dose_dev) {
  int rc = plan_use(P);
  if (rc) return rc;
  if (!x_dev || !G_out) return set_error(IMRT_EINVAL, "x or G_out is NULL");
  const imrt_dose* D = P->dose;
  float* d_int = (dose_dev && D->vox) ? P->vtmp : dose_dev;
  if ((rc = use_device(P->ctx))) return rc;
  // rows the wave blocks skip have no nonzeros: their dose is 0
  if (d_int && !D->gaps.empty() && P->ctx->tune.fwd_wave && (rc = launch_zero(P->ctx, d_int, D->nv))) return rc;
  if ((rc = eval_forward(P, x_dev, d_int, nullptr, 0))) return rc;
  if (dose_dev && D->vox && (rc = launch_permute(P->ctx, P->vtmp, D->vox, D->nv, dose_dev, true))) return rc;
  if ((rc = fetch_misc(P, 1))) return rc;
  *G_out = P->misc_host[0];
  return IMRT_OK;
}

int imrt_gradient(imrt_plan* P, const float* x_dev, float* g_dev, double* G_out) {
  int rc = plan_use(P);
  if (rc) return rc;
  if (!x_dev || !g_dev) return set_error(IMRT_EINVAL, "x or g is NULL");
  if ((rc = use_device(P->ctx)) || (rc = eval_forward(P, x_dev, nullptr, P->rbuf[0], 0)) ||
      (rc = adjoint_into(P->ctx, P->dose, P->rbuf[0], 2.0, g_dev)))
    return rc;
  if (G_out) {
    if ((rc = fetch_misc(P, 1))) return rc;
    *G_out = P->misc_host[0];
  }
  return IMRT_OK;
}

int imrt_gradient_noalloc(imrt_plan* P, const float* x_dev, float* g_dev, double* G_out) {
  int rc = plan_ready(P);
  if (rc) return rc;
  if (!x_dev || !g_dev) return set_error(IMRT_EINVAL, "x or g is NULL");
  if ((rc = use_device(P->ctx))) return rc;
  unsigned char* base = noalloc_scratch(P->ctx->device);
  if (!base) return set_error(IMRT_EINVAL, "no scratch for this device (create the context first)");
  const imrt_dose* D = P->dose;
  const int grid = forward_grid(P->ctx, D, 1);
  // scratch layout, every part 256-byte aligned: residual (nv floats),
  // forward objective partials (grid doubles), adjoint pieces (2 per
  // adjoint workgroup), objective total (one double)
  auto up = [](size_t n) { return (n + 255) & ~static_cast<size_t>(255); };
  const size_t off_r = 0;
  const size_t off_part = off_r + up(sizeof(float) * static_cast<size_t>(D->nv));
  const size_t off_pieces = off_part + up(sizeof(double) * (static_cast<size_t>(grid) + 1));
  const size_t off_total = off_pieces + up(sizeof(double) * 2 * static_cast<size_t>(D->adj_grid));
  const size_t need = off_total + up(sizeof(double));
  if (need > IMRT_NOALLOC_SCRATCH_BYTES)
    return set_error(IMRT_EINVAL, "imrt_gradient_noalloc: the plan needs " + std::to_string(need) +
                                      " bytes of scratch, more than the " +
                                      std::to_string(static_cast<long long>(IMRT_NOALLOC_SCRATCH_BYTES)) +
                                      " available (about 4 million voxels)");
  float* r = reinterpret_cast<float*>(base + off_r);
  double* parts = reinterpret_cast<double*>(base + off_part);
  double* pieces = reinterpret_cast<double*>(base + off_pieces);
  double* total = reinterpret_cast<double*>(base + off_total);
  // forward pass: residual and objective partials (every workgroup writes its
  // own partial and every row its residual, so nothing starts at zero)
  FwdArgs fa = base_fwd(D);
  fa.mode = FWD_EVAL;
  set_plan_penalties(fa, P);
  fa.x = x_dev;
  fa.r_out = r;
  fa.partials = parts;
  if ((rc = launch_forward(P->ctx, D, fa, 1, grid)) ||
      (rc = launch_sum(P->ctx, parts, grid, total, plan_skip_objective(P))))
    return rc;
  // adjoint pass: g = 2 D^T r (pieces written by the workgroups that share a column)
  AdjArgs aa = base_adj(D);
  aa.solve = 0;
  aa.r = r;
  aa.pieces = pieces;
  aa.out = g_dev;
  aa.scale = 2.0;
  if ((rc = launch_adjoint(P->ctx, D, aa, 1))) return rc;
  if (G_out) {
    IMRT_HIP(hipMemcpyAsync(P->misc_host, total, sizeof(double), hipMemcpyDeviceToHost, P->ctx->stream));
    IMRT_HIP(hipStreamSynchronize(P->ctx->stream));
    *G_out = P->misc_host[0];
  }
  return IMRT_OK;
}

int imrt_project(imrt_plan* P, const float* x_dev, const float* g_dev, double lambda, float* x_out_dev,
                 double* step_sq_out) {
  if (!P || !x_dev || !g_dev || !x_out_dev) return set_error(IMRT_EINVAL, "plan, x, g or x_out is NULL");
  if (!std::isfinite(lambda) || lambda < 0) return set_error(IMRT_EINVAL, "lambda must be finite and >= 0");
  int rc;
  if ((rc = use_device(P->ctx)) ||
      (rc = launch_project(P->ctx, x_dev, g_dev, lambda, P->dose->nb, x_out_dev, P->misc)))
    return rc;
  if (step_sq_out) {
    if ((rc = fetch_misc(P, 1))) return rc;
    *step_sq_out = P->misc_host[0];
  }
  return IMRT_OK;
}

int imrt_estimate_lambda0(imrt_plan* P, const float* v0_dev, int32_t iters, double* lambda0_out,
                          double* sigma_out) {
  int rc = plan_use(P);
  if (rc) return rc;
  if (!v0_dev || iters < 0) return set_error(IMRT_EINVAL, "v0 is NULL or iters < 0");
  if ((rc = use_device(P->ctx))) return rc;
  const imrt_dose* D = P->dose;
  const imrt_ctx* C = P->ctx;
  float* v = P->xbuf[0];
  float* w = P->gk;
  if ((rc = launch_normalize(C, v0_dev, D->nb, v, P->misc + 1))) return rc;
  for (int it = 0; it <= iters; ++it) {
    FwdArgs a = base_fwd(D);
    a.mode = FWD_PLAIN;
    a.x = v;
    a.d_out = P->vtmp;
    a.partials = P->fwd_partials;
    const int grid = std::min(forward_grid(C, D), P->fwd_cap);
    if ((rc = launch_forward(C, D, a, 1, grid))) return rc;
    if (it == iters) {
      if ((rc = launch_sum(C, P->fwd_partials, grid, P->misc))) return rc;
      break;
    }
    if ((rc = adjoint_into(C, D, P->vtmp, 1.0, w))) return rc;
    if ((rc = launch_normalize(C, w, D->nb, v, P->misc + 1))) return rc;
  }
  if ((rc = fetch_misc(P, 2))) return rc;
  const double s2 = P->misc_host[0];
  if (P->misc_host[1] == 0.0 || !(s2 > 0.0)) return set_error(IMRT_EINVAL, "power iteration reached a zero vector");
  if (!(P->w_max > 0.0)) return set_error(IMRT_EINVAL, "all penalty weights are zero");
  const double L = 2.0 * P->w_max * s2;
  if (lambda0_out) *lambda0_out = pow2_at_least(2.0 / L);
  if (sigma_out) *sigma_out = std::sqrt(s2);
  return IMRT_OK;
}

// Trace entries of a resumed solve continue the numbering of the solve it
// resumes.
void number_trace(const imrt_solve_params* prm, int n) {
  if (!prm->resume) return;
  auto* t = static_cast<imrt_trace_entry*>(prm->trace);
  for (int i = 0; i < n; ++i) t[i].k += prm->k0;
}

// Checks of a solve's arguments, x_1 >= 0 (host copy), the plan's buffers and
// trace, and the initial solver state.
int solve_prepare(imrt_plan* P, const imrt_solve_params* prm, const float* x_dev, int* nt_out, int* cap_out,
                  SolverState* init_out) {
  int rc = plan_use(P);
  if (rc) return rc;
  if (!prm || !x_dev) return set_error(IMRT_EINVAL, "params or x is NULL");
  if (!(prm->eps > 0.0 && prm->eps < 1.0)) return set_error(IMRT_EINVAL, "eps must lie in (0, 1)");
  if (!(prm->alpha > 1.0) || !std::isfinite(prm->alpha)) return set_error(IMRT_EINVAL, "alpha must be > 1");
  if (!(prm->lambda0 > 0.0) || !std::isfinite(prm->lambda0)) return set_error(IMRT_EINVAL, "lambda0 must be > 0");
  if (!(prm->delta >= 0.0)) return set_error(IMRT_EINVAL, "delta must be >= 0");
  if (prm->max_iter < 0 || prm->max_backtracks < 0)
    return set_error(IMRT_EINVAL, "max_iter and max_backtracks must be >= 0");
  if (prm->warm_start != 0 && prm->warm_start != 1) return set_error(IMRT_EINVAL, "warm_start must be 0 or 1");
  if (prm->profile < 0) return set_error(IMRT_EINVAL, "profile must be >= 0");
  if (prm->resume != 0 && prm->resume != 1) return set_error(IMRT_EINVAL, "resume must be 0 or 1");
  if (prm->resume) {
    if (prm->k0 < 1) return set_error(IMRT_EINVAL, "a resumed solve needs k0 >= 1");
    if (!(prm->G_prev >= 0.0) || !std::isfinite(prm->G_prev))
      return set_error(IMRT_EINVAL, "a resumed solve needs a finite G_prev >= 0");
    if (!(prm->lambda_prev > 0.0) || !std::isfinite(prm->lambda_prev))
      return set_error(IMRT_EINVAL, "a resumed solve needs a finite lambda_prev > 0");
  }
  const int nt = prm->trials_per_pass == 0 ? 1 : prm->trials_per_pass;
  if (nt != 1 && nt != 2 && nt != 4) return set_error(IMRT_EINVAL, "trials_per_pass must be 0, 1, 2 or 4");
  if ((rc = use_device(P->ctx))) return rc;
  const imrt_dose* D = P->dose;
  imrt_ctx* C = P->ctx;
  hipStream_t s = C->stream;
  if (forward_lds_bytes(D->nb, nt, P->nstruct, C->tune.fwd_wave != 0, D->fwd_st, D->fwd_waves) > C->max_lds)
    return set_error(IMRT_EUNSUPPORTED, "nb * trials_per_pass exceeds the LDS budget of the forward pass");

  // x_1 >= 0 and finite (initialisation of the method)
  std::vector<float> xh(D->nb);
  IMRT_HIP(hipMemcpyAsync(xh.data(), x_dev, sizeof(float) * D->nb, hipMemcpyDeviceToHost, s));
  IMRT_HIP(hipStreamSynchronize(s));
  for (float v : xh)
    if (!(v >= 0.0f) || !std::isfinite(v)) return set_error(IMRT_EINVAL, "x_1 must be finite and >= 0");
  if ((rc = ensure_buffers(P, nt + 1))) return rc;
  // the iterate buffers other than x_1's start zeroed (the forward pass
  // blends all candidates with 0/1 weights, so none may be non-finite)
  for (int j = 1; j <= nt; ++j) IMRT_HIP(hipMemsetAsync(P->xbuf[j], 0, sizeof(float) * D->nb, s));
  const int cap = prm->trace ? prm->max_iter : 0;
  if (cap > P->trace_cap) {
    dev_free(P->trace);
    P->trace_cap = 0;
    if ((rc = dev_alloc(&P->trace, cap))) return rc;
    P->trace_cap = cap;
  }
  SolverState init{};
  init.phase = PH_INIT;
  init.status = IMRT_MAX_ITER;
  init.acc = 0;
  init.xi = 0;
  init.ntrials = nt;
  init.max_iter = prm->max_iter;
  init.max_bt = prm->max_backtracks;
  init.fixed = prm->fixed_iters ? 1 : 0;
  init.trace_cap = cap;
  init.warm = prm->warm_start;
  init.resume = prm->resume;
  init.G_prev = prm->resume ? prm->G_prev : 0.0;
  // first trial step: step 2's lambda0, or after a resumed warm-started
  // iteration alpha times the step accepted last (the product the decision
  // forms on the device)
  init.lambda = (prm->resume && prm->warm_start) ? prm->alpha * prm->lambda_prev : prm->lambda0;
  init.eps = prm->eps;
  init.alpha = prm->alpha;
  init.lambda0 = prm->lambda0;
  init.delta = prm->delta;
  *nt_out = nt;
  *cap_out = cap;
  *init_out = init;
  return IMRT_OK;
}

// The forward and adjoint arguments of a plan's solve passes (without the
// state pointers, which depend on the pass).
void solve_args(imrt_plan* P, int nt, int grid, int cap, FwdArgs& fa, AdjArgs& aa) {
  const imrt_dose* D = P->dose;
  fa = base_fwd(D);
  fa.mode = FWD_SOLVE;
  fa.grid = grid;
  set_plan_penalties(fa, P);
  fa.g = P->gk;
  fa.col_kind = D->col_kind;
  fa.pieces_col = P->pieces_col;
  fa.pieces = P->pieces;
  fa.col_wlo = D->col_wlo;
  fa.col_whi = D->col_whi;
  fa.g_scale = 2.0;
  for (int i = 0; i <= kMaxTrials; ++i) {
    fa.xbuf[i] = P->xbuf[i];
    fa.rbuf[i] = P->rbuf[i];
  }
  fa.partials = P->fwd_partials;
  aa = base_adj(D);
  aa.solve = 1;
  for (int i = 0; i <= kMaxTrials; ++i) aa.rbuf[i] = P->rbuf[i];
  aa.pieces = P->pieces;
  aa.pieces_col = P->pieces_col;
  aa.out = P->gk;
  aa.scale = 2.0;
  aa.fwd_partials = P->fwd_partials;
  aa.fwd_parts = grid;
  aa.step_partials = P->fwd_partials + static_cast<size_t>(nt) * grid;
  aa.step_parts = 1;
  aa.trace = cap > 0 ? P->trace : nullptr;
  aa.G_skip = plan_skip_objective(P);
}

int imrt_solve(imrt_plan* P, const imrt_solve_params* prm, float* x_dev, imrt_solve_result* res) {
  if (!res) return set_error(IMRT_EINVAL, "result is NULL");
  int nt = 1, cap = 0, rc;
  SolverState init{};
  if ((rc = solve_prepare(P, prm, x_dev, &nt, &cap, &init))) return rc;
  const imrt_dose* D = P->dose;
  imrt_ctx* C = P->ctx;
  hipStream_t s = C->stream;
  P->st_host[0] = init;

  hipEvent_t ev_start = nullptr, ev_end = nullptr, ev_poll[2] = {nullptr, nullptr};
  // profile mode: HIP events around every profile-th forward and adjoint launch
  struct Timed {
    long long launch;
    hipEvent_t a, b;
  };
  std::vector<Timed> ev_fwd, ev_adj;
  long long n_fwd_launch = 0, n_adj_launch = 0;
  auto cleanup = [&]() {
    if (ev_start) (void)hipEventDestroy(ev_start);
    if (ev_end) (void)hipEventDestroy(ev_end);
    for (auto& e : ev_poll)
      if (e) (void)hipEventDestroy(e);
    for (auto* pool : {&ev_fwd, &ev_adj})
      for (auto& t : *pool) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
      }
  };
  auto event_pair = [&](std::vector<Timed>& pool, long long& launch, hipEvent_t* a, hipEvent_t* b) -> hipError_t {
    *a = *b = nullptr;
    const long long idx = launch++;
    if (prm->profile == 0 || idx % prm->profile != 0) return hipSuccess;
    hipEvent_t x = nullptr, y = nullptr;
    hipError_t r = hipEventCreate(&x);
    if (r == hipSuccess) r = hipEventCreate(&y);
    if (r != hipSuccess) {
      if (x) (void)hipEventDestroy(x);
      return r;
    }
    pool.push_back(Timed{idx, x, y});
    *a = x;
    *b = y;
    return hipSuccess;
  };
  hipError_t e = hipEventCreate(&ev_start);
  if (e == hipSuccess) e = hipEventCreate(&ev_end);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_poll[0], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_poll[1], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev_start, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->st, &P->st_host[0], sizeof(SolverState), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->st + 1, &P->st_host[0], sizeof(SolverState), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->xbuf[0], x_dev, sizeof(float) * D->nb, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    cleanup();
    return hip_error(e, "solve setup");
  }

  const int grid = std::min(forward_grid(C, D, nt), P->fwd_cap);
  FwdArgs fa;
  AdjArgs aa;
  solve_args(P, nt, grid, cap, fa, aa);

  // The two state copies alternate: pass n reads st[n % 2] and writes st[(n + 1) % 2].
  long long pass = 0;
  auto state_in = [&]() { return P->st + (pass & 1); };
  auto state_out = [&]() { return P->st + ((pass + 1) & 1); };
  auto forward_pass = [&]() -> int {
    hipEvent_t f0, f1;
    const hipError_t r = event_pair(ev_fwd, n_fwd_launch, &f0, &f1);
    if (r != hipSuccess) return hip_error(r, "hipEventCreate");
    fa.st_in = state_in();
    fa.st_out = state_out();
    const int rr = launch_forward(C, D, fa, nt, grid, f0, f1);
    ++pass;
    return rr;
  };
  auto adjoint_pass = [&]() -> int {
    hipEvent_t a0, a1;
    const hipError_t r = event_pair(ev_adj, n_adj_launch, &a0, &a1);
    if (r != hipSuccess) return hip_error(r, "hipEventCreate");
    aa.st_in = state_in();
    aa.st_out = state_out();
    const int rr = launch_adjoint(C, D, aa, nt, a0, a1);
    ++pass;
    return rr;
  };

  // initial evaluation G(x_1)
  if ((rc = forward_pass())) {
    (void)hipStreamSynchronize(s);
    cleanup();
    return rc;
  }
  // Iterations are enqueued in batches of (adjoint, forward) groups: each
  // adjoint pass first decides on the forward pass before it.
  // After each batch a copy of the device state is queued; the host waits on
  // the older of two outstanding copies, so one batch is always in flight and
  // the device never waits for the host.  Groups enqueued after convergence
  // exit at once.
  const long long max_groups =
      (static_cast<long long>(prm->max_iter) + 1) * (prm->max_backtracks / nt + 2) + 4;
  struct Poll {
    int slot;
    long long enq;
  };
  Poll q[2];
  int nq = 0, next_slot = 0;
  long long enq = 0, enq_seen = 0;
  int k_seen = 0;
  for (;;) {
    long long batch = C->tune.batch_iters;
    if (prm->fixed_iters) {
      const long long need = static_cast<long long>(prm->max_iter) - k_seen - (enq - enq_seen);
      batch = std::max(0LL, std::min(batch, need));
      if (batch == 0 && nq == 0) batch = 1;
    }
    if (batch > 0 && nq < 2) {
      for (long long i = 0; i < batch; ++i) {
        if ((rc = adjoint_pass()) || (rc = forward_pass())) {
          (void)hipStreamSynchronize(s);
          cleanup();
          return rc;
        }
      }
      enq += batch;
      const int slot = next_slot;
      next_slot ^= 1;
      e = hipMemcpyAsync(&P->st_host[slot], state_in(), sizeof(SolverState), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipEventRecord(ev_poll[slot], s);
      if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        cleanup();
        return hip_error(e, "solve poll");
      }
      q[nq++] = Poll{slot, enq};
    } else {
      batch = 0;
    }
    if (nq == 2 || (batch == 0 && nq > 0)) {
      const Poll p = q[0];
      q[0] = q[1];
      --nq;
      e = hipEventSynchronize(ev_poll[p.slot]);
      if (e != hipSuccess) {
        cleanup();
        return hip_error(e, "solve poll wait");
      }
      const SolverState seen = P->st_host[p.slot];
      k_seen = seen.k;
      enq_seen = p.enq;
      if (seen.phase == PH_DONE) break;
    }
    if (enq > max_groups) {
      (void)hipStreamSynchronize(s);
      cleanup();
      return set_error(IMRT_EINVAL, "internal: solver state machine did not terminate");
    }
  }
  // final state and iterate
  e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(&P->st_host[0], state_in(), sizeof(SolverState), hipMemcpyDeviceToHost);
  const int xi = P->st_host[0].xi;
  if (e == hipSuccess && (xi < 0 || xi > nt)) {
    cleanup();
    return set_error(IMRT_EINVAL, "internal: iterate buffer index out of range");
  }
  if (e == hipSuccess) e = hipMemcpyAsync(x_dev, P->xbuf[xi], sizeof(float) * D->nb, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(ev_end, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev_start, ev_end);
  if (e != hipSuccess) {
    cleanup();
    return hip_error(e, "solve finish");
  }
  const SolverState done_st = P->st_host[0];
  res->iterations = done_st.k;
  res->forward_passes = done_st.n_fwd;
  res->adjoint_passes = done_st.n_adj;
  res->status = done_st.status;
  res->G_initial = done_st.G_init;
  res->G_final = done_st.G;
  res->device_ms = ms;
  res->forward_kernel_ms = 0.0;
  res->adjoint_kernel_ms = 0.0;
  if (prm->profile) {
    // mean over the sampled launches among those that did work
    auto mean_of = [&](const std::vector<Timed>& pool, int n, double* out) -> hipError_t {
      double tot = 0.0;
      int cnt = 0;
      for (const Timed& t : pool) {
        if (t.launch >= n) break;
        float ms_i = 0.f;
        const hipError_t r = hipEventElapsedTime(&ms_i, t.a, t.b);
        if (r != hipSuccess) return r;
        tot += ms_i;
        ++cnt;
      }
      *out = cnt > 0 ? tot / cnt : 0.0;
      return hipSuccess;
    };
    e = mean_of(ev_fwd, done_st.n_fwd, &res->forward_kernel_ms);
    if (e == hipSuccess) e = mean_of(ev_adj, done_st.n_adj, &res->adjoint_kernel_ms);
    if (e != hipSuccess) {
      cleanup();
      return hip_error(e, "kernel timing");
    }
  }
  if (prm->trace && done_st.k > 0) {
    const int n = std::min(done_st.k, cap);
    e = hipMemcpy(prm->trace, P->trace, sizeof(TraceDev) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      cleanup();
      return hip_error(e, "trace copy");
    }
    number_trace(prm, n);
  }
  cleanup();
  return IMRT_OK;
}

int imrt_plan_destroy(imrt_plan* plan) {
  free_plan(plan);
  return IMRT_OK;
}

}  // extern "C"

// ---- batched solve -----------------------------------------------------------------
namespace {

// Slot table of the plans in `active`: each plan's workgroups in order,
// starting at a multiple of the die count (padding slots idle).
void batch_slots(const std::vector<int>& active, const std::vector<int>& grids, std::vector<int32_t>& slots) {
  slots.clear();
  for (int i : active) {
    while (slots.size() % kXcds) slots.push_back(-1);
    for (int w = 0; w < grids[i]; ++w) slots.push_back((i << 16) | w);
  }
}

struct BatchBuffers {
  SolverState* st = nullptr;      // 2 per plan: [2i] read by forward passes, [2i+1] by adjoint passes
  FwdArgs* fargs = nullptr;
  AdjArgs* aargs = nullptr;
  int32_t* fslots = nullptr;
  int32_t* aslots = nullptr;
  SolverState* poll = nullptr;    // pinned host, 2 slots of 2n states
  hipEvent_t ev_start = nullptr, ev_end = nullptr, ev_poll[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // graphs replaced while a launch of theirs may still be queued; destroyed
  // with the buffers, after the batch's stream has drained (the stream guard
  // of imrt_solve_batch is destroyed first and synchronises it)
  std::vector<hipGraphExec_t> old_exec;
  std::vector<hipGraph_t> old_graph;
  ~BatchBuffers() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipGraphExec_t x : old_exec) (void)hipGraphExecDestroy(x);
    for (hipGraph_t g : old_graph) (void)hipGraphDestroy(g);
    for (hipEvent_t e : {ev_start, ev_end, ev_poll[0], ev_poll[1]})
      if (e) (void)hipEventDestroy(e);
    if (poll) (void)hipHostFree(poll);
    for (void* p : {static_cast<void*>(st), static_cast<void*>(fargs), static_cast<void*>(aargs),
                    static_cast<void*>(fslots), static_cast<void*>(aslots)})
      if (p) (void)hipFree(p);
  }
};

}  // namespace

int imrt_solve_batch(int32_t n, imrt_plan* const* plans, const imrt_solve_params* params, float* const* x_dev,
                     imrt_solve_result* results) {
  if (n <= 0 || n > 32767 || !plans || !params || !x_dev || !results)
    return set_error(IMRT_EINVAL, "n must be in [1, 32767]; plans, params, x and results must not be NULL");
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return set_error(IMRT_EINVAL, "a plan is NULL");
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return set_error(IMRT_EINVAL, "a plan appears twice in the batch");
  }
  imrt_ctx* C = plans[0]->ctx;
  for (int i = 0; i < n; ++i) {
    if (plans[i]->ctx != C) return set_error(IMRT_EINVAL, "all plans of a batch must share one context");
    if (plans[i]->dose && (plans[i]->dose->storage != plans[0]->dose->storage ||
                           plans[i]->dose->fwd_st != plans[0]->dose->fwd_st ||
                           plans[i]->dose->fwd_waves != plans[0]->dose->fwd_waves))
      return set_error(IMRT_EINVAL,
                       "all dose matrices of a batch must have the same storage, layout and forward workgroup size "
                       "(partition them alike, e.g. with imrt_dose_repartition_targets)");
  }
  if (C->tune.fwd_wave == 0) return set_error(IMRT_EUNSUPPORTED, "the batched solve needs fwd_wave = 1");
  std::vector<int> nt(n), cap(n), fgrid(n), agrid(n);
  std::vector<SolverState> init(n);
  int rc;
  for (int i = 0; i < n; ++i) {
    if ((rc = solve_prepare(plans[i], &params[i], x_dev[i], &nt[i], &cap[i], &init[i]))) return rc;
    if (nt[i] != nt[0]) return set_error(IMRT_EINVAL, "all plans of a batch must use the same trials_per_pass");
    if (plans[i]->dose->adj_grid >= 65536) return set_error(IMRT_EUNSUPPORTED, "adjoint grid too large for a batch");
  }
  const int storage = plans[0]->dose->storage, fst = plans[0]->dose->fwd_st, fwv = plans[0]->dose->fwd_waves;
  BatchBuffers B;
  // The batch runs on a stream of its own (a graph cannot be captured on the
  // null stream), ordered after the work already on the context's stream;
  // the context's stream is restored on return, after the batch finished.
  struct StreamSwap {
    imrt_ctx* C = nullptr;
    hipStream_t user = nullptr, own = nullptr;
    hipEvent_t ready = nullptr;
    ~StreamSwap() {
      if (own) {
        (void)hipStreamSynchronize(own);
        (void)hipStreamDestroy(own);
      }
      if (ready) (void)hipEventDestroy(ready);
      if (C) C->stream = user;
    }
  } swap;
  swap.user = C->stream;
  IMRT_HIP(hipStreamCreateWithFlags(&swap.own, hipStreamNonBlocking));
  IMRT_HIP(hipEventCreateWithFlags(&swap.ready, hipEventDisableTiming));
  IMRT_HIP(hipEventRecord(swap.ready, swap.user));
  IMRT_HIP(hipStreamWaitEvent(swap.own, swap.ready, 0));
  swap.C = C;
  C->stream = swap.own;
  hipStream_t s = C->stream;
  std::vector<FwdArgs> fa(n);
  std::vector<AdjArgs> aa(n);
  size_t lds = 0;
  for (int i = 0; i < n; ++i) {
    imrt_plan* P = plans[i];
    fgrid[i] = std::min(forward_grid(C, P->dose, nt[i]), P->fwd_cap);
    agrid[i] = P->dose->adj_grid;
    lds = std::max(lds, forward_lds_bytes(P->dose->nb, nt[i], P->nstruct, true, fst, fwv));
  }
  // the live plans' matrix streams share the last-level cache: their policy
  // follows the bytes of the distinct matrices of the unfinished plans
  // together, taken again whenever plans drop out
  auto live_policy = [&](const std::vector<int>& live) {
    std::vector<const imrt_dose*> seen;
    int64_t bytes = 0;
    for (int i : live)
      if (std::find(seen.begin(), seen.end(), plans[i]->dose) == seen.end()) {
        seen.push_back(plans[i]->dose);
        bytes += stream_bytes(plans[i]->dose);
      }
    return stream_policy(C, bytes);
  };
  int batch_cp = 0;
  if (dev_alloc(&B.st, 2 * static_cast<size_t>(n)) || dev_alloc(&B.fargs, n) || dev_alloc(&B.aargs, n))
    return IMRT_ENOMEM;
  for (int i = 0; i < n; ++i) {
    solve_args(plans[i], nt[i], fgrid[i], cap[i], fa[i], aa[i]);
    fa[i].st_in = B.st + 2 * i;
    fa[i].st_out = B.st + 2 * i + 1;
    aa[i].st_in = B.st + 2 * i + 1;
    aa[i].st_out = B.st + 2 * i;
  }
  std::vector<int> active(n);
  for (int i = 0; i < n; ++i) active[i] = i;
  batch_cp = live_policy(active);
  std::vector<int32_t> fs, as;
  batch_slots(active, fgrid, fs);
  batch_slots(active, agrid, as);
  if (dev_alloc(&B.fslots, fs.size()) || dev_alloc(&B.aslots, as.size())) return IMRT_ENOMEM;
  std::vector<SolverState> st_host(2 * static_cast<size_t>(n));
  for (int i = 0; i < n; ++i) st_host[2 * i] = st_host[2 * i + 1] = init[i];
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&B.poll), sizeof(SolverState) * 4 * n, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreate(&B.ev_start);
  if (e == hipSuccess) e = hipEventCreate(&B.ev_end);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B.ev_poll[0], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B.ev_poll[1], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(B.ev_start, s);
  if (e == hipSuccess) e = hipMemcpyAsync(B.st, st_host.data(), sizeof(SolverState) * 2 * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(B.fargs, fa.data(), sizeof(FwdArgs) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(B.aargs, aa.data(), sizeof(AdjArgs) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(B.fslots, fs.data(), sizeof(int32_t) * fs.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(B.aslots, as.data(), sizeof(int32_t) * as.size(), hipMemcpyHostToDevice, s);
  for (int i = 0; i < n && e == hipSuccess; ++i)
    e = hipMemcpyAsync(plans[i]->xbuf[0], x_dev[i], sizeof(float) * plans[i]->dose->nb, hipMemcpyDeviceToDevice, s);
  // the host vectors above must outlive the copies
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "batch setup");

  // initial evaluation G(x_1) of every plan
  if ((rc = launch_forward_batch(C, B.fargs, B.fslots, static_cast<int>(fs.size()), nt[0], fst, fwv, lds, batch_cp))) {
    (void)hipStreamSynchronize(s);
    return rc;
  }
  // Batches of (adjoint, forward) groups over the active plans, captured
  // once per set of active plans as a graph and replayed; the host polls a
  // copy of every plan's state one batch behind and drops finished plans
  // from the slot tables (stream-ordered uploads, then a new capture).
  const long long K = C->tune.batch_iters;
  auto capture = [&]() -> int {
    batch_cp = live_policy(active);
    // the previous graph may still have a launch queued: keep it until the end
    if (B.exec) B.old_exec.push_back(B.exec);
    if (B.graph) B.old_graph.push_back(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
    hipError_t r = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (r != hipSuccess) return hip_error(r, "hipStreamBeginCapture");
    int lrc = IMRT_OK;
    for (long long k = 0; k < K && lrc == IMRT_OK; ++k) {
      lrc = launch_adjoint_batch(C, B.aargs, B.aslots, static_cast<int>(as.size()), nt[0], storage, batch_cp);
      if (lrc == IMRT_OK)
        lrc = launch_forward_batch(C, B.fargs, B.fslots, static_cast<int>(fs.size()), nt[0], fst, fwv, lds, batch_cp);
    }
    r = hipStreamEndCapture(s, &B.graph);
    if (lrc) return lrc;
    if (r != hipSuccess) return hip_error(r, "hipStreamEndCapture");
    r = hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0);
    if (r != hipSuccess) return hip_error(r, "hipGraphInstantiate");
    return IMRT_OK;
  };
  if ((rc = capture())) {
    (void)hipStreamSynchronize(s);
    return rc;
  }
  long long max_groups = 4;
  for (int i = 0; i < n; ++i)
    max_groups = std::max(max_groups, (static_cast<long long>(params[i].max_iter) + 1) *
                                          (params[i].max_backtracks / nt[i] + 2) + 4);
  // slot tables whose stream-ordered uploads may still be pending
  std::vector<std::vector<int32_t>> keep;
  keep.reserve(4 * static_cast<size_t>(n) + 4);
  int q[2];
  int nq = 0, next_slot = 0;
  long long enq = 0;
  for (;;) {
    const bool launch = !active.empty() && nq < 2;
    if (launch) {
      e = hipGraphLaunch(B.exec, s);
      const int slot = next_slot;
      next_slot ^= 1;
      if (e == hipSuccess)
        e = hipMemcpyAsync(B.poll + 2 * static_cast<size_t>(n) * slot, B.st, sizeof(SolverState) * 2 * n,
                           hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipEventRecord(B.ev_poll[slot], s);
      if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        return hip_error(e, "batch launch");
      }
      enq += K;
      q[nq++] = slot;
    }
    if (nq == 2 || (!launch && nq > 0)) {
      const int slot = q[0];
      q[0] = q[1];
      --nq;
      e = hipEventSynchronize(B.ev_poll[slot]);
      if (e != hipSuccess) return hip_error(e, "batch poll wait");
      const SolverState* seen = B.poll + 2 * static_cast<size_t>(n) * slot;
      std::vector<int> still;
      for (int i : active)
        if (seen[2 * i + 1].phase != PH_DONE) still.push_back(i);
      if (still.size() != active.size()) {
        active.swap(still);
        if (!active.empty()) {
          // (each table stays in `keep` until the end: its upload is asynchronous)
          keep.emplace_back();
          batch_slots(active, fgrid, keep.back());
          const std::vector<int32_t>& nf = keep.back();
          e = hipMemcpyAsync(B.fslots, nf.data(), sizeof(int32_t) * nf.size(), hipMemcpyHostToDevice, s);
          fs.assign(nf.begin(), nf.end());
          keep.emplace_back();
          batch_slots(active, agrid, keep.back());
          const std::vector<int32_t>& na = keep.back();
          if (e == hipSuccess)
            e = hipMemcpyAsync(B.aslots, na.data(), sizeof(int32_t) * na.size(), hipMemcpyHostToDevice, s);
          as.assign(na.begin(), na.end());
          if (e != hipSuccess) {
            (void)hipStreamSynchronize(s);
            return hip_error(e, "batch slot upload");
          }
          if ((rc = capture())) {
            (void)hipStreamSynchronize(s);
            return rc;
          }
        }
      }
    }
    if (active.empty() && nq == 0) break;
    if (enq > max_groups) {
      (void)hipStreamSynchronize(s);
      return set_error(IMRT_EINVAL, "internal: batched state machines did not terminate");
    }
  }
  e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(st_host.data(), B.st, sizeof(SolverState) * 2 * n, hipMemcpyDeviceToHost);
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    const int xi = st_host[2 * i + 1].xi;
    if (xi < 0 || xi > nt[i]) return set_error(IMRT_EINVAL, "internal: iterate buffer index out of range");
    e = hipMemcpyAsync(x_dev[i], plans[i]->xbuf[xi], sizeof(float) * plans[i]->dose->nb, hipMemcpyDeviceToDevice, s);
  }
  if (e == hipSuccess) e = hipEventRecord(B.ev_end, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, B.ev_start, B.ev_end);
  if (e != hipSuccess) return hip_error(e, "batch finish");
  for (int i = 0; i < n; ++i) {
    const SolverState& f = st_host[2 * i + 1];
    imrt_solve_result& r = results[i];
    r.iterations = f.k;
    r.forward_passes = f.n_fwd;
    r.adjoint_passes = f.n_adj;
    r.status = f.status;
    r.G_initial = f.G_init;
    r.G_final = f.G;
    r.device_ms = ms;
    r.forward_kernel_ms = 0.0;
    r.adjoint_kernel_ms = 0.0;
    if (params[i].trace && f.k > 0) {
      const int m = std::min(f.k, cap[i]);
      e = hipMemcpy(params[i].trace, plans[i]->trace, sizeof(TraceDev) * m, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_error(e, "trace copy");
      number_trace(&params[i], m);
    }
  }
  return IMRT_OK;
}

namespace {
// A new work partition (and forward workgroup size) for a dose matrix.
int repartition(imrt_dose* D, int32_t adj_min_nnz, int32_t fwd_blocks_per_wave, int32_t fwd_waves) {
  if (!D) return set_error(IMRT_EINVAL, "dose is NULL");
  if (adj_min_nnz < 16 || fwd_blocks_per_wave < 1 || fwd_blocks_per_wave > 1024)
    return set_error(IMRT_EINVAL, "adj_min_nnz must be >= 16 and fwd_blocks_per_wave in [1, 1024]");
  int rc = use_device(D->ctx);
  if (rc) return rc;
  hipStream_t s = D->ctx->stream;
  IMRT_HIP(hipStreamSynchronize(s));
  if (adj_min_nnz == D->adj_min_nnz && fwd_blocks_per_wave == D->fwd_bpw && fwd_waves == D->fwd_waves) return IMRT_OK;
  try {
    std::vector<int32_t> rp(static_cast<size_t>(D->nv) + 1), cp(static_cast<size_t>(D->nb) + 1);
    IMRT_HIP(hipMemcpy(rp.data(), D->row_ptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost));
    IMRT_HIP(hipMemcpy(cp.data(), D->col_ptr, sizeof(int32_t) * cp.size(), hipMemcpyDeviceToHost));
    D->adj_min_nnz = adj_min_nnz;
    D->fwd_bpw = fwd_blocks_per_wave;
    D->fwd_waves = fwd_waves;
    return finish_dose(D, rp, cp);
  } catch (const std::bad_alloc&) {
    return set_error(IMRT_ENOMEM, "host allocation failed");
  }
}
}  // namespace

int imrt_dose_repartition(imrt_dose* D, int32_t adj_min_nnz, int32_t fwd_blocks_per_wave) {
  if (!D) return set_error(IMRT_EINVAL, "dose is NULL");
  return repartition(D, adj_min_nnz, fwd_blocks_per_wave, D->fwd_waves);
}

// Per-plan targets serve dispatches that several plans share: their forward
// workgroups have 8 waves (see partition_for_targets).
int imrt_dose_repartition_targets(imrt_dose* D, int32_t adj_workgroups, int32_t fwd_workgroups) {
  if (!D) return set_error(IMRT_EINVAL, "dose is NULL");
  if (adj_workgroups < 1 || fwd_workgroups < 1) return set_error(IMRT_EINVAL, "workgroup targets must be >= 1");
  int32_t a = 0, b = 0;
  partition_for_targets(D->nnz, adj_workgroups, fwd_workgroups, &a, &b);
  return repartition(D, a, b, 8);
}

int imrt_dose_partition(const imrt_dose* D, int32_t* adj_min_nnz, int32_t* fwd_blocks_per_wave) {
  if (!D) return set_error(IMRT_EINVAL, "dose is NULL");
  if (adj_min_nnz) *adj_min_nnz = D->adj_min_nnz;
  if (fwd_blocks_per_wave) *fwd_blocks_per_wave = D->fwd_bpw;
  return IMRT_OK;
}

// Launch-shape search for a batch: every candidate (fewest nonzeros per
// adjoint workgroup, row blocks per forward wave) is applied to all the
// batch's dose matrices, and a short batched solve (tune_iters fixed
// iterations from the given x, on copies) is timed by stream events; the
// fastest candidate is left applied.
int imrt_batch_autotune(int32_t n, imrt_plan* const* plans, const imrt_solve_params* params,
                        const float* const* x_dev, int32_t tune_iters, int32_t* ta_out, int32_t* tf_out) {
  if (n <= 0 || !plans || !params || !x_dev || tune_iters < 0)
    return set_error(IMRT_EINVAL, "n must be positive, tune_iters >= 0; plans, params and x must not be NULL");
  for (int i = 0; i < n; ++i)
    if (!plans[i] || !plans[i]->dose) return set_error(IMRT_EINVAL, "a plan is NULL or has no dose matrix");
  std::vector<imrt_dose*> doses;
  for (int i = 0; i < n; ++i) {
    imrt_dose* d = const_cast<imrt_dose*>(plans[i]->dose);
    if (std::find(doses.begin(), doses.end(), d) == doses.end()) doses.push_back(d);
  }
  int rc = use_device(plans[0]->ctx);
  if (rc) return rc;
  // working copies of the start points and tuning parameters
  std::vector<float*> xs(n, nullptr);
  auto release = [&]() {
    for (float*& p : xs) dev_free(p);
  };
  for (int i = 0; i < n; ++i) {
    if ((rc = dev_alloc(&xs[i], plans[i]->dose->nb))) {
      release();
      return rc;
    }
  }
  std::vector<imrt_solve_params> prm(params, params + n);
  for (auto& p : prm) {
    if (tune_iters > 0) {
      p.max_iter = tune_iters;
      p.fixed_iters = 1;
    }
    p.trace = nullptr;
    p.profile = 0;
  }
  std::vector<imrt_solve_result> res(n);
  // Candidates are per-plan targets: about `ta` adjoint workgroups and `tf`
  // forward workgroups per plan, i.e. for a matrix of nnz nonzeros
  // nnz / ta nonzeros per adjoint workgroup (within [1024, 32768]) and
  // nnz / (8 tf kWaveNnz) row blocks per forward wave (8-wave workgroups;
  // within [1, 4]).  Few
  // workgroups per plan spend less on their starts while many plans share a
  // dispatch; many keep a plan fast once it runs alone.
  struct Cand {
    int32_t ta, tf;
  };
  const Cand cands[] = {{32, 16}, {128, 32}, {128, 128}, {512, 64}, {512, 256}, {2048, 512}};
  auto part_of = [](const imrt_dose* d, const Cand& c, int32_t* a, int32_t* b) {
    partition_for_targets(d->nnz, c.ta, c.tf, a, b);
  };
  double best = -1.0;
  Cand best_c = cands[0];
  hipStream_t s = plans[0]->ctx->stream;
  for (const Cand& c : cands) {
    for (imrt_dose* d : doses) {
      int32_t a = 0, b = 0;
      part_of(d, c, &a, &b);
      if ((rc = repartition(d, a, b, 8))) {
        release();
        return rc;
      }
    }
    for (int i = 0; i < n; ++i) {
      const hipError_t e = hipMemcpyAsync(xs[i], x_dev[i], sizeof(float) * plans[i]->dose->nb,
                                          hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) {
        release();
        return hip_error(e, "autotune copy");
      }
    }
    if ((rc = imrt_solve_batch(n, plans, prm.data(), xs.data(), res.data()))) {
      release();
      return rc;
    }
    const double ms = res[0].device_ms;
    if (best < 0.0 || ms < best) {
      best = ms;
      best_c = c;
    }
  }
  release();
  for (imrt_dose* d : doses) {
    int32_t a = 0, b = 0;
    part_of(d, best_c, &a, &b);
    if ((rc = repartition(d, a, b, 8))) return rc;
  }
  if (ta_out) *ta_out = best_c.ta;
  if (tf_out) *tf_out = best_c.tf;
  return IMRT_OK;
}
