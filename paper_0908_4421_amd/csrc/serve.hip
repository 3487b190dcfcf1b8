// Re-plan server: requests arrive at any time and are admitted by HBM
// footprint into one set of live solves whose iterations run batched
// (continuous batching: a request joins the running dispatches at the next
// poll, a finished one leaves them), with every dose matrix, plan and solver
// state resident on the device.  Each solve computes what imrt_solve
// computes alone, since the batched passes keep every plan's own work
// partition and reduction order.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <mutex>
#include <thread>
#include <vector>

#include "imrt_internal.h"

// Shared with imrt_solve (api.hip, which defines them with C linkage).
extern "C" {
int solve_prepare(imrt_plan* P, const imrt_solve_params* prm, const float* x_dev, int* nt_out, int* cap_out,
                  imrt::SolverState* init_out);
void solve_args(imrt_plan* P, int nt, int grid, int cap, imrt::FwdArgs& fa, imrt::AdjArgs& aa);
}

using namespace imrt;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Pending {
  int64_t ticket;
  int64_t patient;
  bool have_geometry;
  imrt_geometry geometry;
  int storage;
  std::vector<imrt_penalty> penalties;
  double x0;
  imrt_solve_params params;
  Clock::time_point arrival;
};

struct Resident {
  imrt_dose* dose = nullptr;
  int64_t bytes = 0;
  int users = 0;
  uint64_t last_use = 0;
};

struct Live {
  int64_t ticket = 0;
  int64_t patient = 0;
  imrt_plan* plan = nullptr;
  float* x = nullptr;          // start point, then scratch
  int64_t bytes = 0;           // plan buffers charged to the budget
  int nt = 1, grid = 1;
  Clock::time_point arrival, admitted;
  double lambda0 = 0.0;
  void* trace_dst = nullptr;   // the request's trace buffer (filled by its wait)
  int trace_cap = 0;
  int32_t resume = 0, k0 = 0;
};

struct Finished {
  imrt_solve_result result{};
  imrt_serve_times times{};
  std::vector<float> x;
  int rc = IMRT_OK;
  std::string error;
  std::vector<imrt_trace_entry> trace;   // accepted iterations, numbered as in imrt_solve
  void* trace_dst = nullptr;
};

// Device bytes of a dose matrix (values, indices, partition tables) and of a
// plan's buffers, as allocated by this library.
int64_t dose_bytes(const imrt_dose* D) {
  const int64_t nnz = D->nnz, nv = D->nv, nb = D->nb;
  const int64_t per_nz = (D->storage == ST_F32) ? (D->col16 ? 18 : 16) : 10;
  return per_nz * nnz + 4 * (nv + 1) + 4 * (nb + 1) + 2 * nv /* ids, order */ + 4 * nv /* permutation scratch */ +
         4 * static_cast<int64_t>(D->nwblocks + D->nblocks) * 2 + 16 * D->adj_grid + 9 * nb;
}

int64_t plan_bytes(const imrt_dose* D, int nt) {
  const int64_t nv = D->nv, nb = D->nb;
  return (4 * (nt + 1) + 4 + 1) * nv + (4 * (nt + 1) + 4 + 16) * nb + 16 * D->adj_grid + 8 * 4096;
}

}  // namespace

struct imrt_server {
  imrt_ctx* user = nullptr;
  imrt_ctx ctx;                 // the server's own stream on the user's device
  int64_t budget = 0, used = 0, peak = 0, reserve = 0;
  int max_live = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Pending> queue;
  std::map<int64_t, Finished> finished;
  std::set<int64_t> delivered;  // tickets already handed to a waiter
  std::map<int64_t, Resident> residents;
  uint64_t use_clock = 0;
  int64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  // device-side batch tables (capacity max_live plans)
  SolverState* st = nullptr;
  FwdArgs* fargs = nullptr;
  AdjArgs* aargs = nullptr;
  int32_t* fslots = nullptr;
  int32_t* aslots = nullptr;
  int32_t* gtab = nullptr;      // shared-matrix adjoint groups
  size_t fslot_cap = 0, aslot_cap = 0, gtab_cap = 0;
  int64_t shared_groups = 0;    // adjoint dispatch groups that served two or more solves at once
  int64_t adj_groups = 0;       // adjoint dispatch groups in all
  std::vector<Live> live;       // index = batch slot of the plan
  std::vector<char> occupied;
  int64_t served = 0;
  std::string fatal;
};

namespace {

constexpr size_t kShareMax = 4;   // solves per shared-matrix adjoint group

int grow_slots(imrt_server* S, int32_t** p, size_t* cap, size_t need) {
  if (need <= *cap) return IMRT_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(int32_t) * std::max<size_t>(need, 1024));
  if (e != hipSuccess) return hip_error(e, "hipMalloc(server slots)");
  *cap = std::max<size_t>(need, 1024);
  (void)S;
  return IMRT_OK;
}

// Evict resident matrices nobody uses, least recently used first, until
// `need` more bytes fit the budget (caller holds no lock; worker only).
bool make_room(imrt_server* S, int64_t need) {
  while (S->used + need > S->budget) {
    auto victim = S->residents.end();
    for (auto it = S->residents.begin(); it != S->residents.end(); ++it)
      if (it->second.users == 0 && (victim == S->residents.end() || it->second.last_use < victim->second.last_use))
        victim = it;
    if (victim == S->residents.end()) return false;
    (void)imrt_dose_destroy(victim->second.dose);
    S->used -= victim->second.bytes;
    S->residents.erase(victim);
  }
  return true;
}

void finish_error(imrt_server* S, int64_t ticket, int rc, const Pending* p) {
  Finished f;
  f.rc = rc;
  f.error = imrt_last_error();
  if (p) f.times.queue_ms = ms_between(p->arrival, Clock::now());
  std::lock_guard<std::mutex> g(S->mu);
  S->finished[ticket] = std::move(f);
  S->cv_done.notify_all();
}

// Admit one request into a free batch slot: resident or new dose matrix,
// plan, structures and penalties, lambda_0 if not given, start point, the
// initial evaluation pass.  Returns false when it must wait for memory.
bool admit(imrt_server* S, Pending& p, int slot) {
  imrt_ctx* C = &S->ctx;
  int rc;
  // dose matrix
  auto rit = S->residents.find(p.patient);
  imrt_dose* D = nullptr;
  if (rit != S->residents.end()) {
    D = rit->second.dose;
  } else {
    if (!p.have_geometry) {
      finish_error(S, p.ticket, set_error(IMRT_EINVAL, "patient not resident and no geometry given"), &p);
      return true;
    }
    if (!make_room(S, S->reserve)) return false;
    if ((rc = imrt_build_dose_matrix(C, &p.geometry, static_cast<imrt_dtype>(p.storage), &D, nullptr))) {
      finish_error(S, p.ticket, rc, &p);
      return true;
    }
    Resident r;
    r.dose = D;
    r.bytes = dose_bytes(D);
    S->reserve = std::max(S->reserve, r.bytes);
    if (!make_room(S, r.bytes)) {   // larger than foreseen: wait until it fits
      (void)imrt_dose_destroy(D);
      return false;
    }
    S->used += r.bytes;
    S->peak = std::max(S->peak, S->used);
    rit = S->residents.emplace(p.patient, r).first;
  }
  const int nt = p.params.trials_per_pass == 0 ? 1 : p.params.trials_per_pass;
  // One dispatch serves one storage, forward layout and trial count: a
  // request that differs from the live solves waits until they are done.
  for (int i = 0; i < S->max_live; ++i) {
    if (!S->occupied[i]) continue;
    const imrt_dose* LD = S->live[i].plan->dose;
    if (LD->storage != D->storage || LD->fwd_st != D->fwd_st || LD->fwd_waves != D->fwd_waves || S->live[i].nt != nt)
      return false;
  }
  const int64_t pb = plan_bytes(D, nt) + (p.params.trace ? static_cast<int64_t>(sizeof(imrt_trace_entry)) *
                                                              std::max(0, p.params.max_iter) : 0);
  if (S->used + pb > S->budget) {
    rit->second.users += 1;   // keep it while making room for the plan
    const bool ok = make_room(S, pb);
    rit->second.users -= 1;
    if (!ok) return false;
  }
  Live L;
  L.ticket = p.ticket;
  L.patient = p.patient;
  L.arrival = p.arrival;
  L.bytes = pb;
  auto fail = [&](int code) {
    if (L.plan) (void)imrt_plan_destroy(L.plan);
    if (L.x) (void)hipFree(L.x);
    finish_error(S, p.ticket, code, &p);
    return true;
  };
  if ((rc = imrt_plan_create(C, D, &L.plan))) return fail(rc);
  if ((rc = imrt_set_structures(L.plan, nullptr, static_cast<int32_t>(p.penalties.size())))) return fail(rc);
  if ((rc = imrt_set_penalties(L.plan, p.penalties.data()))) return fail(rc);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&L.x), sizeof(float) * D->nb);
  if (e != hipSuccess) return fail(hip_error(e, "hipMalloc(start point)"));
  std::vector<float> xh(D->nb, static_cast<float>(p.x0));
  if (p.params.lambda0 <= 0.0) {
    // lambda_0 from 50 power iterations started at the all-ones vector
    std::vector<float> ones(D->nb, 1.0f);
    e = hipMemcpy(L.x, ones.data(), sizeof(float) * D->nb, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(hip_error(e, "upload"));
    double lam = 0.0;
    if ((rc = imrt_estimate_lambda0(L.plan, L.x, 50, &lam, nullptr))) return fail(rc);
    p.params.lambda0 = lam;
  }
  L.lambda0 = p.params.lambda0;
  e = hipMemcpy(L.x, xh.data(), sizeof(float) * D->nb, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(hip_error(e, "upload"));
  int cap = 0;
  SolverState init{};
  p.params.profile = 0;
  if ((rc = solve_prepare(L.plan, &p.params, L.x, &L.nt, &cap, &init))) return fail(rc);
  if (S->ctx.tune.fwd_wave == 0) return fail(set_error(IMRT_EUNSUPPORTED, "serving needs fwd_wave = 1"));
  L.grid = std::min(forward_grid(C, D, L.nt), L.plan->fwd_cap);
  FwdArgs fa;
  AdjArgs aa;
  solve_args(L.plan, L.nt, L.grid, cap, fa, aa);
  L.trace_dst = p.params.trace;
  L.trace_cap = cap;
  L.resume = p.params.resume;
  L.k0 = p.params.k0;
  fa.st_in = S->st + 2 * slot;
  fa.st_out = S->st + 2 * slot + 1;
  aa.st_in = S->st + 2 * slot + 1;
  aa.st_out = S->st + 2 * slot;
  hipStream_t s = C->stream;
  const SolverState two[2] = {init, init};
  e = hipMemcpyAsync(S->st + 2 * slot, two, sizeof(two), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(S->fargs + slot, &fa, sizeof(fa), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(S->aargs + slot, &aa, sizeof(aa), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(L.plan->xbuf[0], L.x, sizeof(float) * D->nb, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(hip_error(e, "admission upload"));
  // the initial evaluation G(x_1), alone (the batch then continues with
  // (adjoint, forward) groups)
  if ((rc = launch_forward(C, D, fa, L.nt, L.grid))) return fail(rc);
  e = hipStreamSynchronize(s);   // the small host arrays above must outlive the copies
  if (e != hipSuccess) return fail(hip_error(e, "admission"));
  L.admitted = Clock::now();
  rit->second.users += 1;
  rit->second.last_use = ++S->use_clock;
  S->used += pb;
  S->peak = std::max(S->peak, S->used);
  S->live[slot] = L;
  S->occupied[slot] = 1;
  return true;
}

void release(imrt_server* S, int slot) {
  Live& L = S->live[slot];
  (void)imrt_plan_destroy(L.plan);
  if (L.x) (void)hipFree(L.x);
  S->used -= L.bytes;
  auto it = S->residents.find(L.patient);
  if (it != S->residents.end()) it->second.users -= 1;
  L = Live{};
  S->occupied[slot] = 0;
}

void worker_main(imrt_server* S) {
  (void)hipSetDevice(S->ctx.device);
  imrt_ctx* C = &S->ctx;
  hipStream_t s = C->stream;
  const int K = std::max(1, S->ctx.tune.serve_groups);   // groups between polls: bounds a new request's wait
  std::vector<SolverState> seen(2 * static_cast<size_t>(S->max_live));
  std::vector<int32_t> fs, as, gt;
  for (;;) {
    // admission, in arrival order, while a slot and memory are free
    std::vector<Pending> take;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      const bool idle = std::none_of(S->occupied.begin(), S->occupied.end(), [](char c) { return c != 0; });
      if (idle && S->queue.empty()) {
        if (S->stop) break;
        S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
        if (S->stop && S->queue.empty()) break;
      }
      int free_slots = 0;
      for (char c : S->occupied) free_slots += (c == 0);
      while (free_slots-- > 0 && !S->queue.empty()) {
        take.push_back(S->queue.front());
        S->queue.pop_front();
      }
    }
    std::vector<Pending> back;   // requests that must wait for memory
    bool changed = false;
    for (Pending& p : take) {
      if (!back.empty()) {   // keep arrival order behind a waiting request
        back.push_back(p);
        continue;
      }
      int slot = 0;
      while (S->occupied[slot]) ++slot;
      if (admit(S, p, slot)) {
        changed = changed || S->occupied[slot];
      } else {
        back.push_back(p);
      }
    }
    if (!back.empty()) {
      std::lock_guard<std::mutex> g(S->mu);
      for (auto it = back.rbegin(); it != back.rend(); ++it) S->queue.push_front(*it);
    }
    std::vector<int> active;
    for (int i = 0; i < S->max_live; ++i)
      if (S->occupied[i]) active.push_back(i);
    if (active.empty()) {
      if (!back.empty()) {
        // nothing live and the head does not fit even after eviction
        Pending p;
        {
          std::lock_guard<std::mutex> g(S->mu);
          p = S->queue.front();
          S->queue.pop_front();
        }
        finish_error(S, p.ticket, set_error(IMRT_ENOMEM, "request does not fit the HBM budget"), &p);
      }
      continue;
    }
    // slot tables of the live plans (each at a multiple of the die count)
    fs.clear();
    as.clear();
    gt.clear();
    int storage = -1, fst = -1, fwv = 16, nt = 1;
    size_t lds = 0;
    bool mixed = false;
    for (int i : active) {
      const Live& L = S->live[i];
      const imrt_dose* D = L.plan->dose;
      if (storage < 0) {
        storage = D->storage;
        fst = D->fwd_st;
        fwv = D->fwd_waves;
        nt = L.nt;
      }
      mixed = mixed || D->storage != storage || D->fwd_st != fst || D->fwd_waves != fwv || L.nt != nt;
      while (fs.size() % kXcds) fs.push_back(-1);
      for (int w = 0; w < L.grid; ++w) fs.push_back((i << 16) | w);
      lds = std::max(lds, forward_lds_bytes(D->nb, L.nt, L.plan->nstruct, true, D->fwd_st, D->fwd_waves));
    }
    // Adjoint slots: the live solves on one resident matrix (re-plans of a
    // patient) form groups of up to kShareMax that read the matrix once per
    // pass (shared-matrix adjoint); without sharing every solve is its own
    // group.  Each group takes the matrix's adjoint grid of slots.
    std::vector<std::vector<int>> groups;
    {
      std::vector<const imrt_dose*> order;
      std::map<const imrt_dose*, std::vector<int>> by_dose;
      for (int i : active) {
        const imrt_dose* D = S->live[i].plan->dose;
        if (!S->ctx.tune.serve_shared_adj) {
          groups.push_back({i});
          continue;
        }
        if (!by_dose.count(D)) order.push_back(D);
        by_dose[D].push_back(i);
      }
      for (const imrt_dose* D : order) {
        const std::vector<int>& v = by_dose[D];
        for (size_t j = 0; j < v.size(); j += kShareMax)
          groups.emplace_back(v.begin() + j, v.begin() + std::min(v.size(), j + kShareMax));
      }
    }
    size_t gmax = 1;
    for (const auto& g : groups) gmax = std::max(gmax, g.size());
    const int gk = gmax <= 1 ? 1 : (gmax <= 2 ? 2 : 4);
    for (size_t g = 0; g < groups.size(); ++g) {
      const imrt_dose* D = S->live[groups[g][0]].plan->dose;
      const int id = (gk == 1) ? groups[g][0] : static_cast<int>(g);
      while (as.size() % kXcds) as.push_back(-1);
      for (int w = 0; w < D->adj_grid; ++w) as.push_back((id << 16) | w);
      if (gk > 1) {
        gt.push_back(static_cast<int32_t>(groups[g].size()));
        for (int q = 0; q < gk; ++q) gt.push_back(groups[g][std::min<size_t>(q, groups[g].size() - 1)]);
      }
    }
    int rc = IMRT_OK;
    if (mixed) rc = set_error(IMRT_EINVAL, "live solves of one server must share storage, layout and trials_per_pass");
    if (!rc) rc = grow_slots(S, &S->fslots, &S->fslot_cap, fs.size());
    if (!rc) rc = grow_slots(S, &S->aslots, &S->aslot_cap, as.size());
    if (!rc && gk > 1) rc = grow_slots(S, &S->gtab, &S->gtab_cap, gt.size());
    hipError_t e = hipSuccess;
    if (!rc) e = hipMemcpyAsync(S->fslots, fs.data(), sizeof(int32_t) * fs.size(), hipMemcpyHostToDevice, s);
    if (!rc && e == hipSuccess)
      e = hipMemcpyAsync(S->aslots, as.data(), sizeof(int32_t) * as.size(), hipMemcpyHostToDevice, s);
    if (!rc && e == hipSuccess && gk > 1)
      e = hipMemcpyAsync(S->gtab, gt.data(), sizeof(int32_t) * gt.size(), hipMemcpyHostToDevice, s);
    if (!rc && e != hipSuccess) rc = hip_error(e, "server slot upload");
    for (int k = 0; k < K && !rc; ++k) {
      if (gk == 1) rc = launch_adjoint_batch(C, S->aargs, S->aslots, static_cast<int>(as.size()), nt, storage, 0);
      else
        rc = launch_adjoint_multi_batch(C, S->aargs, S->gtab, gk, S->aslots, static_cast<int>(as.size()), nt,
                                        storage);
      if (!rc) rc = launch_forward_batch(C, S->fargs, S->fslots, static_cast<int>(fs.size()), nt, fst, fwv, lds, 0);
    }
    if (!rc) {
      std::lock_guard<std::mutex> g(S->mu);
      S->adj_groups += static_cast<int64_t>(K) * static_cast<int64_t>(groups.size());
      for (const auto& grp : groups) S->shared_groups += (grp.size() > 1) ? K : 0;
    }
    if (!rc) {
      e = hipMemcpyAsync(seen.data(), S->st, sizeof(SolverState) * 2 * S->max_live, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) rc = hip_error(e, "server poll");
    }
    if (rc) {
      // a failed dispatch fails every live request
      for (int i : active) {
        finish_error(S, S->live[i].ticket, rc, nullptr);
        release(S, i);
      }
      continue;
    }
    (void)changed;
    for (int i : active) {
      const SolverState& f = seen[2 * i + 1];
      if (f.phase != PH_DONE) continue;
      Live& L = S->live[i];
      Finished out;
      out.result.iterations = f.k;
      out.result.forward_passes = f.n_fwd;
      out.result.adjoint_passes = f.n_adj;
      out.result.status = f.status;
      out.result.G_initial = f.G_init;
      out.result.G_final = f.G;
      const imrt_dose* D = L.plan->dose;
      out.x.resize(D->nb);
      e = hipMemcpy(out.x.data(), L.plan->xbuf[f.xi], sizeof(float) * D->nb, hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        out.rc = hip_error(e, "result copy");
        out.error = imrt_last_error();
      }
      const Clock::time_point now = Clock::now();
      out.times.queue_ms = ms_between(L.arrival, L.admitted);
      out.times.plan_ms = ms_between(L.arrival, now);
      out.times.lambda0 = L.lambda0;
      out.times.nnz = D->nnz;
      out.times.nv = D->nv;
      out.times.nb = D->nb;
      if (L.trace_dst && f.k > 0 && out.rc == IMRT_OK) {
        out.trace.resize(std::min(f.k, L.trace_cap));
        e = hipMemcpy(out.trace.data(), L.plan->trace, sizeof(imrt_trace_entry) * out.trace.size(),
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
          out.rc = hip_error(e, "trace copy");
          out.error = imrt_last_error();
        }
        if (L.resume)
          for (auto& t : out.trace) t.k += L.k0;
        out.trace_dst = L.trace_dst;
      }
      const int64_t ticket = L.ticket;   // (release clears the slot's record)
      release(S, i);
      std::lock_guard<std::mutex> g(S->mu);
      S->finished[ticket] = std::move(out);
      S->served += 1;
      S->cv_done.notify_all();
    }
  }
}

}  // namespace

int imrt_server_create(imrt_ctx* ctx, int64_t hbm_budget_bytes, int32_t max_live, imrt_server** out) {
  if (!ctx || !out) return set_error(IMRT_EINVAL, "ctx or out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes <= 0 || max_live <= 0 || max_live > 4096)
    return set_error(IMRT_EINVAL, "budget must be positive and max_live in [1, 4096]");
  IMRT_HIP(hipSetDevice(ctx->device));
  auto* S = new (std::nothrow) imrt_server();
  if (!S) return set_error(IMRT_ENOMEM, "host allocation failed");
  S->user = ctx;
  S->ctx = *ctx;
  S->ctx.stream = nullptr;
  // matrices the server builds take per-plan partition targets: few
  // workgroups for a large plan sharing its dispatches, enough for a small
  // one to run fast when it is (nearly) alone
  S->ctx.tune.part_adj_wgs = ctx->tune.serve_adj_wgs;
  S->ctx.tune.part_fwd_wgs = ctx->tune.serve_fwd_wgs;
  S->budget = hbm_budget_bytes;
  S->reserve = std::min<int64_t>(hbm_budget_bytes / 2, int64_t(1) << 28);
  S->max_live = max_live;
  S->live.resize(max_live);
  S->occupied.assign(max_live, 0);
  hipError_t e = hipStreamCreateWithFlags(&S->ctx.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->st), sizeof(SolverState) * 2 * max_live);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->fargs), sizeof(FwdArgs) * max_live);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->aargs), sizeof(AdjArgs) * max_live);
  if (e == hipSuccess) {
    // idle slots read as finished
    std::vector<SolverState> done(2 * static_cast<size_t>(max_live));
    for (auto& x : done) x.phase = PH_DONE;
    e = hipMemcpy(S->st, done.data(), sizeof(SolverState) * done.size(), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    const int rc = hip_error(e, "server setup");
    if (S->st) (void)hipFree(S->st);
    if (S->fargs) (void)hipFree(S->fargs);
    if (S->aargs) (void)hipFree(S->aargs);
    if (S->ctx.stream) (void)hipStreamDestroy(S->ctx.stream);
    delete S;
    return rc;
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return IMRT_OK;
}

int imrt_server_submit(imrt_server* S, const imrt_request* r, int64_t* ticket_out) {
  if (!S || !r || !ticket_out) return set_error(IMRT_EINVAL, "server, request or ticket is NULL");
  if (!r->penalties || r->nstruct <= 0 || r->nstruct > kMaxStruct)
    return set_error(IMRT_EINVAL, "penalties must hold 1..256 structures");
  if (r->storage != IMRT_F32 && r->storage != IMRT_BF16 && r->storage != IMRT_F16)
    return set_error(IMRT_EINVAL, "unknown storage");
  if (!(r->x0 >= 0.0) || !std::isfinite(r->x0)) return set_error(IMRT_EINVAL, "x0 must be finite and >= 0");
  Pending p;
  p.patient = r->patient;
  p.have_geometry = r->geometry != nullptr;
  if (r->geometry) p.geometry = *r->geometry;
  p.storage = r->storage;
  p.penalties.assign(r->penalties, r->penalties + r->nstruct);
  p.x0 = r->x0;
  p.params = r->params;
  p.arrival = Clock::now();
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) return set_error(IMRT_EINVAL, "server is shutting down");
  p.ticket = S->next_ticket++;
  S->queue.push_back(p);
  *ticket_out = p.ticket;
  S->cv_work.notify_all();
  return IMRT_OK;
}

int imrt_server_wait(imrt_server* S, int64_t ticket, float* x_out, int32_t nb, imrt_solve_result* result,
                     imrt_serve_times* times, int64_t timeout_ms) {
  if (!S) return set_error(IMRT_EINVAL, "server is NULL");
  if (timeout_ms <= 0) return set_error(IMRT_EINVAL, "timeout_ms must be positive");
  Finished f;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    if (ticket <= 0 || ticket >= S->next_ticket) return set_error(IMRT_EINVAL, "unknown ticket");
    if (S->delivered.count(ticket)) return set_error(IMRT_EINVAL, "ticket already handed out or being waited on");
    S->delivered.insert(ticket);   // (a second waiter on the same ticket is turned away)
    const bool ready = S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                                           [&] { return S->finished.count(ticket) != 0; });
    if (!ready) {
      S->delivered.erase(ticket);  // still pending: a later wait may collect it
      return set_error(IMRT_ETIMEDOUT, "ticket " + std::to_string(ticket) + " not finished after " +
                                           std::to_string(timeout_ms) + " ms");
    }
    Finished& done = S->finished[ticket];
    if (x_out && done.rc == IMRT_OK && nb != static_cast<int32_t>(done.x.size())) {
      S->delivered.erase(ticket);  // the result stays for a wait with the right length
      return set_error(IMRT_EINVAL, "x_out length differs from nb");
    }
    f = std::move(done);
    S->finished.erase(ticket);
  }
  if (f.rc) return set_error(f.rc, f.error);
  if (x_out) std::memcpy(x_out, f.x.data(), sizeof(float) * f.x.size());
  if (result) *result = f.result;
  if (times) *times = f.times;
  if (f.trace_dst && !f.trace.empty())
    std::memcpy(f.trace_dst, f.trace.data(), sizeof(imrt_trace_entry) * f.trace.size());
  return IMRT_OK;
}

int imrt_server_stats(imrt_server* S, int64_t* used_bytes, int64_t* peak_bytes, int64_t* resident_matrices,
                      int64_t* served) {
  if (!S) return set_error(IMRT_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> g(S->mu);
  if (used_bytes) *used_bytes = S->used;
  if (peak_bytes) *peak_bytes = S->peak;
  if (resident_matrices) *resident_matrices = static_cast<int64_t>(S->residents.size());
  if (served) *served = S->served;
  return IMRT_OK;
}

int imrt_server_adjoint_groups(imrt_server* S, int64_t* shared, int64_t* total) {
  if (!S) return set_error(IMRT_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> g(S->mu);
  if (shared) *shared = S->shared_groups;
  if (total) *total = S->adj_groups;
  return IMRT_OK;
}

int imrt_server_destroy(imrt_server* S) {
  if (!S) return IMRT_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  (void)hipSetDevice(S->ctx.device);
  for (int i = 0; i < S->max_live; ++i)
    if (S->occupied[i]) release(S, i);
  for (auto& kv : S->residents) (void)imrt_dose_destroy(kv.second.dose);
  for (void* p : {static_cast<void*>(S->st), static_cast<void*>(S->fargs), static_cast<void*>(S->aargs),
                  static_cast<void*>(S->fslots), static_cast<void*>(S->aslots), static_cast<void*>(S->gtab)})
    if (p) (void)hipFree(p);
  if (S->ctx.stream) (void)hipStreamDestroy(S->ctx.stream);
  delete S;
  return IMRT_OK;
}
