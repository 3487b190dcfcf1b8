// Hot-path kernels of the gradient-projection / Armijo solver for gfx950.
//
//  fwd_kernel       trial update + projection (step 2/4), forward dose z = D x
//                   over CSR (Section 2.1), penalty residual and objective
//                   partials (Eq. (1)-(2)) fused in one pass over D.
//  adj_chunk_kernel beamlet-parallel adjoint D^T r over CSC, columns split
//                   into fixed nonzero chunks; fixed-order float64 sums.
//  adj_final_kernel per-column sum of the chunk partials, times 2 (gradient).
//  decide_kernel    one workgroup: objective reduction, Armijo test (Eq. (5)),
//                   stopping test (step 5), iterate update, trace.
//
// Every reduction runs in a fixed order, so results are bit-reproducible run
// to run and independent of which workgroup finishes first; there are no
// floating-point atomics.
#include <cmath>

#include "imrt_internal.h"

namespace imrt {
namespace {

// Trial point of steps 2/4: max(0, x - lambda g), evaluated in float64 and
// rounded once to float32.  NaN propagates (it is not clipped to zero).
__device__ __forceinline__ float trial_point(float x, float g, double lam) {
#pragma clang fp contract(off)
  const double t = static_cast<double>(x) - lam * static_cast<double>(g);
  return static_cast<float>(t < 0.0 ? 0.0 : t);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum of v over the workgroup in a fixed order; the result is valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T t = T(0);
  if (threadIdx.x == 0) {
    t = sh[0];
#pragma unroll
    for (int i = 1; i < kWaves; ++i) t += sh[i];
  }
  __syncthreads();
  return t;
}

__device__ __forceinline__ float* select_buf(float* const (&b)[kMaxTrials + 1], int i) {
  float* p = b[0];
  p = (i == 1) ? b[1] : p;
  p = (i == 2) ? b[2] : p;
  p = (i == 3) ? b[3] : p;
  p = (i == 4) ? b[4] : p;
  return p;
}

// Lanes cooperating on one row: the largest power of two with lanes*nr <= 256, at most 64.
__device__ __forceinline__ int lanes_per_row(int nr) {
  int L = 64;
  while (L > 1 && L * nr > kThreads) L >>= 1;
  return L;
}

struct RowPenalty {
  double Tu, To, wu, wo;
};

__device__ __forceinline__ RowPenalty row_penalty(const Penalties& p, int row) {
  const PenaltyDev t = p.table[p.sid[row]];
  RowPenalty r{t.T_u, t.T_o, t.w_u, t.w_o};
  if (p.Tu_vox != nullptr) {
    r.Tu = static_cast<double>(p.Tu_vox[row]);
    r.To = static_cast<double>(p.To_vox[row]);
  }
  return r;
}

// One-sided quadratic penalty of a voxel (Eq. (1)) and its half-derivative.
__device__ __forceinline__ void penalty(const RowPenalty& p, float z, double& F, float& r) {
#pragma clang fp contract(off)
  const double zd = static_cast<double>(z);
  const double under = fmin(zd - p.Tu, 0.0);
  const double over = fmax(zd - p.To, 0.0);
  F = p.wu * under * under + p.wo * over * over;
  r = static_cast<float>(p.wu * under + p.wo * over);
}

template <int NT>
__device__ __forceinline__ void row_epilogue(const FwdArgs& a, int row, const float (&d)[NT],
                                             double (&pacc)[NT], float* const (&rout)[NT], int ntr) {
  if (a.mode == FWD_PLAIN) {
    a.d_out[row] = d[0];
    pacc[0] += static_cast<double>(d[0]) * static_cast<double>(d[0]);
    return;
  }
  const RowPenalty p = row_penalty(a.pen, row);
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    if (q < ntr) {
      double F;
      float r;
      penalty(p, d[q], F, r);
      pacc[q] += F;
      if (a.mode == FWD_SOLVE) {
        rout[q][row] = r;
      } else if (q == 0) {
        if (a.r_out) a.r_out[row] = r;
        if (a.d_out) a.d_out[row] = d[0];
      }
    }
  }
}

// Forward pass.  Each workgroup stages the NT trial vectors
// x_t^(q) = max(0, x_k - lambda_q g_k) in LDS, then walks row blocks of at
// most kFwdNnzMax nonzeros: the block's products D_ij x_t^(q)_i go to LDS with
// fully coalesced loads of col_idx/val, then lanes-per-row groups sum each
// row and the penalty epilogue writes r and accumulates G.
template <int NT>
__global__ __launch_bounds__(kThreads) void fwd_kernel(FwdArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* xs = reinterpret_cast<float*>(smem);
  float* prod = xs + NT * a.nb;
  int32_t* rp = reinterpret_cast<int32_t*>(prod + NT * kFwdNnzMax);
  __shared__ double red[kWaves];
  __shared__ float redf[kWaves];

  const int tid = threadIdx.x;
  const int nb = a.nb;
  int ntr = 1;
  bool direct = true;
  double lam[NT];
  float* rout[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    lam[q] = 0.0;
    rout[q] = nullptr;
  }
  if (a.mode == FWD_SOLVE) {
    const SolverState* st = a.st;
    const int phase = st->phase;
    if (phase == PH_DONE) return;
    direct = (phase == PH_INIT);
    ntr = direct ? 1 : NT;
    const int acc = st->acc;
    lam[0] = st->lambda;
#pragma unroll
    for (int q = 1; q < NT; ++q) lam[q] = lam[q - 1] / st->alpha;
#pragma unroll
    for (int q = 0; q < NT; ++q) rout[q] = select_buf(a.rbuf, (acc + 1 + q) % (NT + 1));
  }

  for (int i = tid; i < nb; i += kThreads) {
    const float xi = a.x[i];
    if (direct) {
#pragma unroll
      for (int q = 0; q < NT; ++q) xs[q * nb + i] = xi;
    } else {
      const float gi = a.g[i];
#pragma unroll
      for (int q = 0; q < NT; ++q) xs[q * nb + i] = trial_point(xi, gi, lam[q]);
    }
  }
  __syncthreads();

  double pacc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) pacc[q] = 0.0;

  for (int b = blockIdx.x; b < a.nblocks; b += gridDim.x) {
    const int r0 = a.block_row[b], r1 = a.block_row[b + 1];
    const int nr = r1 - r0;
    const int k0 = a.row_ptr[r0], k1 = a.row_ptr[r1];
    const int nz = k1 - k0;
    if (nz > kFwdNnzMax) {
      // a single row longer than the LDS block: all lanes stride over it
      float s[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) s[q] = 0.f;
      for (int k = k0 + tid; k < k1; k += kThreads) {
        const int c = a.col_idx[k];
        const float v = a.val[k];
#pragma unroll
        for (int q = 0; q < NT; ++q) s[q] = fmaf(v, xs[q * nb + c], s[q]);
      }
#pragma unroll
      for (int q = 0; q < NT; ++q) s[q] = block_sum(s[q], redf);
      if (tid == 0) row_epilogue<NT>(a, r0, s, pacc, rout, ntr);
      continue;
    }
    for (int k = tid; k < nz; k += kThreads) {
      const int c = a.col_idx[k0 + k];
      const float v = a.val[k0 + k];
#pragma unroll
      for (int q = 0; q < NT; ++q) prod[q * kFwdNnzMax + k] = v * xs[q * nb + c];
    }
    for (int i = tid; i <= nr; i += kThreads) rp[i] = a.row_ptr[r0 + i] - k0;
    __syncthreads();
    const int L = lanes_per_row(nr);
    const int lane = tid & (L - 1);
    for (int row = tid / L; row < nr; row += kThreads / L) {
      const int s0 = rp[row], s1 = rp[row + 1];
      float s[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) s[q] = 0.f;
      for (int k = s0 + lane; k < s1; k += L) {
#pragma unroll
        for (int q = 0; q < NT; ++q) s[q] += prod[q * kFwdNnzMax + k];
      }
      for (int off = L >> 1; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < NT; ++q) s[q] += __shfl_xor(s[q], off, 64);
      }
      if (lane == 0) row_epilogue<NT>(a, r0 + row, s, pacc, rout, ntr);
    }
    __syncthreads();
  }

#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const double t = block_sum(pacc[q], red);
    if (tid == 0) a.partials[q * gridDim.x + blockIdx.x] = t;
  }
}

// Adjoint pass, stage 1: one fixed-order float64 partial per nonzero chunk.
__global__ __launch_bounds__(kThreads) void adj_chunk_kernel(AdjArgs a) {
  const float* r = a.r;
  if (a.solve) {
    if (a.st->phase != PH_NEED_GRAD) return;
    r = select_buf(a.rbuf, a.st->acc);
  }
  __shared__ double red[kWaves];
  const int tid = threadIdx.x;
  for (int c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
    const int k0 = a.chunk_k[c], k1 = a.chunk_k[c + 1];
    double s = 0.0;
    for (int k = k0 + tid; k < k1; k += kThreads)
      s += static_cast<double>(a.val[k]) * static_cast<double>(r[a.row_idx[k]]);
    s = block_sum(s, red);
    if (tid == 0) a.partials[c] = s;
  }
}

// Adjoint pass, stage 2: column sums of the chunk partials, scaled.
__global__ __launch_bounds__(kThreads) void adj_final_kernel(AdjFinalArgs f) {
  if (f.solve && f.st->phase != PH_NEED_GRAD) return;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= f.nb) return;
  double s = 0.0;
  for (int c = f.col_chunk[i]; c < f.col_chunk[i + 1]; ++c) s += f.partials[c];
  f.out[i] = static_cast<float>(f.scale * s);
}

// Line-search decision (one workgroup).
template <int NT>
__global__ __launch_bounds__(kThreads) void decide_kernel(DecideArgs a) {
#pragma clang fp contract(off)
  SolverState* st = a.st;
  const int phase = st->phase;
  if (phase == PH_DONE) return;
  __shared__ double red[kWaves];
  __shared__ double Gq[NT], Sq[NT];
  __shared__ int acc_q;
  __shared__ double acc_lam;
  const int tid = threadIdx.x;
  const bool init = (phase == PH_INIT);
  const int ntr = init ? 1 : NT;
  double lam[NT];
  lam[0] = st->lambda;
#pragma unroll
  for (int q = 1; q < NT; ++q) lam[q] = lam[q - 1] / st->alpha;

#pragma unroll
  for (int q = 0; q < NT; ++q) {
    if (q < ntr) {
      double s = 0.0;
      for (int i = tid; i < a.nparts; i += kThreads) s += a.partials[q * a.nparts + i];
      s = block_sum(s, red);
      if (tid == 0) Gq[q] = s;
    }
  }
  if (!init) {
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      double s = 0.0;
      for (int i = tid; i < a.nb; i += kThreads) {
        const float xi = a.x[i];
        const double dl = static_cast<double>(trial_point(xi, a.g[i], lam[q])) - static_cast<double>(xi);
        s += dl * dl;
      }
      s = block_sum(s, red);
      if (tid == 0) Sq[q] = s;
    }
  }

  if (tid == 0) {
    int accepted = -1;
    double lam_used = lam[0];
    if (init) {
      const double G0 = Gq[0];
      st->n_fwd += 1;
      st->G = G0;
      st->G_init = G0;
      st->G_prev = G0;
      st->acc = (st->acc + 1) % (NT + 1);
      st->m = 0;
      st->lambda = st->lambda0;
      if (!isfinite(G0)) {
        st->status = IMRT_NUMERIC;
        st->phase = PH_DONE;
      } else if (st->max_iter <= 0) {
        st->status = IMRT_MAX_ITER;
        st->phase = PH_DONE;
      } else {
        st->phase = PH_NEED_GRAD;
      }
    } else {
      if (phase == PH_NEED_GRAD) st->n_adj += 1;
      st->n_fwd += 1;
      bool done = false;
      double l = st->lambda;
      for (int q = 0; q < NT; ++q) {
        if (q > 0) l = l / st->alpha;
        lam_used = l;
        const double s = Sq[q], Gt = Gq[q];
        if (s == 0.0) {
          st->status = IMRT_STALLED;
          done = true;
          break;
        }
        if (!isfinite(Gt)) {
          st->status = IMRT_NUMERIC;
          done = true;
          break;
        }
        const double C = st->G - (st->eps / l) * s;   // Eq. (5)
        if (Gt < C) {
          accepted = q;
          break;
        }
        st->m += 1;
        if (st->m > st->max_bt) {
          st->status = IMRT_LS_FAIL;
          done = true;
          break;
        }
      }
      if (accepted >= 0) {
        st->k += 1;
        st->G_prev = st->G;
        st->G = Gq[accepted];
        st->acc = (st->acc + 1 + accepted) % (NT + 1);
        if (a.trace != nullptr && st->k - 1 < st->trace_cap) {
          TraceDev e;
          e.k = st->k;
          e.backtracks = st->m;
          e.lambda = lam_used;
          e.step_sq = Sq[accepted];
          e.G = st->G;
          a.trace[st->k - 1] = e;
        }
        st->m = 0;
        st->lambda = st->lambda0;
        if (st->fixed) {
          if (st->k >= st->max_iter) {
            st->status = IMRT_MAX_ITER;
            done = true;
          }
        } else if (st->G == 0.0 || fabs(st->G - st->G_prev) / st->G < st->delta) {
          st->status = IMRT_CONVERGED;
          done = true;
        } else if (st->k >= st->max_iter) {
          st->status = IMRT_MAX_ITER;
          done = true;
        }
        st->phase = done ? PH_DONE : PH_NEED_GRAD;
      } else if (done) {
        st->phase = PH_DONE;
      } else {
        st->lambda = l / st->alpha;
        st->phase = PH_TRIAL;
      }
    }
    acc_q = init ? -1 : accepted;
    acc_lam = lam_used;
  }
  __syncthreads();
  if (acc_q >= 0) {
    const double l = acc_lam;
    for (int i = tid; i < a.nb; i += kThreads) a.x[i] = trial_point(a.x[i], a.g[i], l);
  }
}

__global__ __launch_bounds__(kThreads) void sum_kernel(const double* parts, int n, double* out) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) s += parts[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(kThreads) void project_kernel(const float* x, const float* g, double lam,
                                                           int nb, float* x_out, double* s_out) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreads) {
    const float xi = x[i];
    const float t = trial_point(xi, g[i], lam);
    x_out[i] = t;
    const double dl = static_cast<double>(t) - static_cast<double>(xi);
    s += dl * dl;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) *s_out = s;
}

__global__ __launch_bounds__(kThreads) void normalize_kernel(const float* w, int nb, float* v,
                                                             double* norm_out) {
  __shared__ double red[kWaves];
  __shared__ double nrm;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreads) {
    const double wi = static_cast<double>(w[i]);
    s += wi * wi;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    nrm = sqrt(s);
    *norm_out = nrm;
  }
  __syncthreads();
  const double n = nrm;
  for (int i = threadIdx.x; i < nb; i += kThreads)
    v[i] = n > 0.0 ? static_cast<float>(static_cast<double>(w[i]) / n) : 0.0f;
}

int check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, what);
  return IMRT_OK;
}

}  // namespace

size_t forward_lds_bytes(int nb, int ntrials) {
  return static_cast<size_t>(ntrials) * (static_cast<size_t>(nb) + kFwdNnzMax) * sizeof(float) +
         static_cast<size_t>(kFwdRowsMax + 1) * sizeof(int32_t);
}

int forward_grid(const imrt_ctx* ctx, const imrt_dose* D) {
  const int cap = ctx->tune.fwd_grid_per_cu * ctx->num_cu;
  return D->nblocks < cap ? (D->nblocks > 0 ? D->nblocks : 1) : cap;
}

int launch_forward(const imrt_ctx* ctx, const imrt_dose* D, const FwdArgs& a, int ntrials, int grid,
                   hipEvent_t before, hipEvent_t after) {
  const size_t lds = forward_lds_bytes(a.nb, ntrials);
  if (lds > ctx->max_lds)
    return set_error(IMRT_EUNSUPPORTED, "forward pass: nb * trials exceeds the LDS budget");
  if (before && hipEventRecord(before, ctx->stream) != hipSuccess) return check_launch("hipEventRecord");
  switch (ntrials) {
    case 1: hipLaunchKernelGGL(fwd_kernel<1>, dim3(grid), dim3(kThreads), lds, ctx->stream, a); break;
    case 2: hipLaunchKernelGGL(fwd_kernel<2>, dim3(grid), dim3(kThreads), lds, ctx->stream, a); break;
    case 4: hipLaunchKernelGGL(fwd_kernel<4>, dim3(grid), dim3(kThreads), lds, ctx->stream, a); break;
    default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
  }
  const int rc = check_launch("fwd_kernel");
  if (rc == IMRT_OK && after && hipEventRecord(after, ctx->stream) != hipSuccess) return check_launch("hipEventRecord");
  return rc;
}

int launch_adjoint(const imrt_ctx* ctx, const imrt_dose* D, const AdjArgs& a, const AdjFinalArgs& f,
                   hipEvent_t before, hipEvent_t after) {
  const int cap = ctx->tune.adj_grid_per_cu * ctx->num_cu;
  const int grid = a.nchunks < cap ? (a.nchunks > 0 ? a.nchunks : 1) : cap;
  if (before && hipEventRecord(before, ctx->stream) != hipSuccess) return check_launch("hipEventRecord");
  hipLaunchKernelGGL(adj_chunk_kernel, dim3(grid), dim3(kThreads), 0, ctx->stream, a);
  int rc = check_launch("adj_chunk_kernel");
  if (rc) return rc;
  if (after && hipEventRecord(after, ctx->stream) != hipSuccess) return check_launch("hipEventRecord");
  const int g2 = (f.nb + kThreads - 1) / kThreads;
  if (g2 > 0) {
    hipLaunchKernelGGL(adj_final_kernel, dim3(g2), dim3(kThreads), 0, ctx->stream, f);
    rc = check_launch("adj_final_kernel");
  }
  return rc;
}

int launch_decide(const imrt_ctx* ctx, const DecideArgs& a, int ntrials) {
  switch (ntrials) {
    case 1: hipLaunchKernelGGL(decide_kernel<1>, dim3(1), dim3(kThreads), 0, ctx->stream, a); break;
    case 2: hipLaunchKernelGGL(decide_kernel<2>, dim3(1), dim3(kThreads), 0, ctx->stream, a); break;
    case 4: hipLaunchKernelGGL(decide_kernel<4>, dim3(1), dim3(kThreads), 0, ctx->stream, a); break;
    default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
  }
  return check_launch("decide_kernel");
}

int launch_sum(const imrt_ctx* ctx, const double* parts, int n, double* out) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kThreads), 0, ctx->stream, parts, n, out);
  return check_launch("sum_kernel");
}

int launch_project(const imrt_ctx* ctx, const float* x, const float* g, double lambda, int nb,
                   float* x_out, double* s_out) {
  hipLaunchKernelGGL(project_kernel, dim3(1), dim3(kThreads), 0, ctx->stream, x, g, lambda, nb, x_out, s_out);
  return check_launch("project_kernel");
}

int launch_normalize(const imrt_ctx* ctx, const float* w, int nb, float* v_out, double* norm_out) {
  hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(kThreads), 0, ctx->stream, w, nb, v_out, norm_out);
  return check_launch("normalize_kernel");
}

}  // namespace imrt
