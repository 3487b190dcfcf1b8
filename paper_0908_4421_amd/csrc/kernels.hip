// Hot-path kernels of the gradient-projection / Armijo solver for gfx950.
//
//  fwd_kernel   trial update + projection (steps 2 and 4) staged in LDS,
//               forward dose z = D x over CSR (Section 2.1), penalty residual
//               and objective partials (Eqs. (1)-(2)), in one pass over D.
//  adj_kernel   line-search decision on the preceding forward pass (Armijo
//               test of Eq. (5), stopping test of step 5), taken identically
//               by every workgroup, then the beamlet-parallel adjoint
//               g = 2 D^T r over CSC for an accepted, unfinished iterate.
//  adj_final    completes beamlet columns shared by several adjoint
//               workgroups (outside a solve, or with the completion not
//               folded into the next forward pass).
//
// The solver state is double-buffered: a pass reads one copy and workgroup 0
// writes the other, so no workgroup ever sees a state written during its own
// pass.  Every reduction runs in a fixed order, so results are
// bit-reproducible and independent of workgroup timing; there are no
// floating-point atomics.  Work is dealt to workgroups in contiguous ranges,
// consecutive ranges on the same accelerator die (workgroups are dispatched
// round-robin over the 8 dies), so neighbouring beamlet columns share that
// die's L2 for their residual gathers.
#include <algorithm>
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

// Contiguous share [begin, end) of n work items for this workgroup.  With a
// grid that is a multiple of the die count, workgroup w (on die w % 8) gets
// logical slot (w % 8) * (grid / 8) + w / 8, so each die owns one contiguous
// eighth of the items.
__device__ __forceinline__ void work_range(int n, int& begin, int& end) {
  const int G = gridDim.x, w = blockIdx.x;
  const int lw = (G % kXcds == 0) ? (w % kXcds) * (G / kXcds) + w / kXcds : w;
  begin = static_cast<int>(static_cast<long long>(lw) * n / G);
  end = static_cast<int>(static_cast<long long>(lw + 1) * n / G);
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

// Penalty of a row: the structure's entry of the LDS copy of the table, or
// per-voxel thresholds when given.
__device__ __forceinline__ RowPenalty row_penalty(const Penalties& p, int row, const PenaltyDev* tab,
                                                  uint8_t sid) {
  const PenaltyDev t = tab[sid];
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
__device__ __forceinline__ void row_epilogue(const FwdArgs& a, int row, uint8_t sid, const PenaltyDev* tab,
                                             const float (&d)[NT], double (&pacc)[NT],
                                             float* const (&rout)[NT], int ntr) {
  if (a.mode == FWD_PLAIN) {
    a.d_out[row] = d[0];
    pacc[0] += static_cast<double>(d[0]) * static_cast<double>(d[0]);
    return;
  }
  const RowPenalty p = row_penalty(a.pen, row, tab, sid);
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

// ---- line-search decision ----------------------------------------------------------
// Decision on the forward pass whose objective partials are in `partials`
// ([trial][nparts], then [trial] step norms), starting from state `in`.  All
// threads of the workgroup take part (fixed-order reductions); the new state
// and the accepted trial land in shared memory.  Every workgroup that runs it
// on the same inputs reaches the same result.
struct Decision {
  SolverState st;   // state after the decision
  int accepted;     // accepted trial, -1 if none
  int backtracks;   // reductions before the accepted trial
  double lam, step_sq;
};

template <int NT>
__device__ void decide(const SolverState* in, const double* partials, int nparts, Decision& dec, double* red) {
#pragma clang fp contract(off)
  __shared__ double Gq[NT];
  const int tid = threadIdx.x;
  if (tid == 0) {
    dec.st = *in;
    dec.accepted = -1;
  }
  __syncthreads();
  if (dec.st.phase == PH_DONE) return;
  const bool init = (dec.st.phase == PH_INIT);
  const int ntr = init ? 1 : NT;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    if (q < ntr) {
      // four independent loads per round, summed in index order
      double s = 0.0;
      const double* pq = partials + q * nparts;
      for (int i0 = tid; i0 < nparts; i0 += 4 * kThreads) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + u * kThreads;
          v[u] = pq[i < nparts ? i : 0];
          v[u] = (i < nparts) ? v[u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s += v[u];
      }
      s = block_sum(s, red);
      if (tid == 0) Gq[q] = s;
    }
  }
  if (tid == 0) {
    SolverState st = dec.st;
    st.n_fwd += 1;
    if (init) {
      const double G0 = Gq[0];
      st.G = G0;
      st.G_init = G0;
      st.G_prev = G0;
      st.acc = (st.acc + 1) % (NT + 1);
      st.m = 0;
      st.lambda = st.lambda0;
      if (!isfinite(G0)) {
        st.status = IMRT_NUMERIC;
        st.phase = PH_DONE;
      } else if (st.max_iter <= 0) {
        st.status = IMRT_MAX_ITER;
        st.phase = PH_DONE;
      } else {
        st.phase = PH_NEED_GRAD;
      }
    } else {
      const double* sq = partials + NT * nparts;
      bool done = false;
      int accepted = -1;
      double l = st.lambda;
      for (int q = 0; q < NT; ++q) {
        if (q > 0) l = l / st.alpha;
        const double s = sq[q], Gt = Gq[q];
        if (s == 0.0) {
          st.status = IMRT_STALLED;
          done = true;
          break;
        }
        if (!isfinite(Gt)) {
          st.status = IMRT_NUMERIC;
          done = true;
          break;
        }
        const double C = st.G - (st.eps / l) * s;   // Eq. (5)
        if (Gt < C) {
          accepted = q;
          break;
        }
        st.m += 1;
        if (st.m > st.max_bt) {
          st.status = IMRT_LS_FAIL;
          done = true;
          break;
        }
      }
      if (accepted >= 0) {
        dec.accepted = accepted;
        dec.backtracks = st.m;
        dec.lam = l;
        dec.step_sq = sq[accepted];
        st.k += 1;
        st.G_prev = st.G;
        st.G = Gq[accepted];
        st.acc = (st.acc + 1 + accepted) % (NT + 1);
        st.xi = (st.xi + 1 + accepted) % (NT + 1);
        st.m = 0;
        st.lambda = st.lambda0;
        if (st.fixed) {
          if (st.k >= st.max_iter) {
            st.status = IMRT_MAX_ITER;
            done = true;
          }
        } else if (st.G == 0.0 || fabs(st.G - st.G_prev) / st.G < st.delta) {
          st.status = IMRT_CONVERGED;
          done = true;
        } else if (st.k >= st.max_iter) {
          st.status = IMRT_MAX_ITER;
          done = true;
        }
        st.phase = done ? PH_DONE : PH_NEED_GRAD;
      } else if (done) {
        st.phase = PH_DONE;
      } else {
        st.lambda = l / st.alpha;
        st.phase = PH_TRIAL;
      }
    }
    if (st.phase == PH_NEED_GRAD) st.n_adj += 1;
    dec.st = st;
  }
  __syncthreads();
}

// ---- forward pass ---------------------------------------------------------------
struct BlockMeta {
  int r0, r1, k0, k1;
};

__device__ __forceinline__ BlockMeta block_meta(const FwdArgs& a, int b) {
  BlockMeta m;
  m.r0 = a.block_row[b];
  m.r1 = a.block_row[b + 1];
  m.k0 = a.block_k0[b];
  m.k1 = a.block_k0[b + 1];
  return m;
}

struct VecRegs {
  int4 c[2];
  float4 v[2];
};

// Issue the 16-byte loads covering nonzeros [base, min(base + 8*256, k1)) of
// an index/value pair of arrays.  base is a multiple of 4 and the arrays carry
// a zeroed tail, so whole vectors stay in bounds; a lane past k1 loads the
// first vector instead (never used), which keeps the loads branch-free.
__device__ __forceinline__ void issue_vec(const int32_t* idx, const float* val, int base, int k1, VecRegs& R) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    int e0 = base + 4 * (threadIdx.x + j * kThreads);
    e0 = (e0 < k1) ? e0 : 0;
    R.c[j] = *reinterpret_cast<const int4*>(idx + e0);
    R.v[j] = *reinterpret_cast<const float4*>(val + e0);
  }
}

// Row pointers (relative to the block's aligned start) and structure ids of
// one block, loaded ahead into registers.
struct RowRegs {
  int rp[3];
  uint8_t sid[2];
};

__device__ __forceinline__ void issue_rows(const FwdArgs& a, const BlockMeta& m, bool want_sid, RowRegs& Q) {
  const int nr = m.r1 - m.r0;
  const int t = threadIdx.x;
  const int i0 = (t <= nr) ? t : 0;
  const int i1 = (t + kThreads <= nr) ? t + kThreads : 0;
  const int i2 = (2 * kThreads <= nr) ? 2 * kThreads : 0;
  Q.rp[0] = a.row_ptr[m.r0 + i0];
  Q.rp[1] = a.row_ptr[m.r0 + i1];
  Q.rp[2] = a.row_ptr[m.r0 + i2];
  if (want_sid) {
    const int j0 = (t < nr) ? t : 0;
    const int j1 = (t + kThreads < nr) ? t + kThreads : 0;
    Q.sid[0] = a.pen.sid[m.r0 + j0];
    Q.sid[1] = a.pen.sid[m.r0 + j1];
  } else {
    Q.sid[0] = Q.sid[1] = 0;
  }
}

__device__ __forceinline__ void stage_rows(const BlockMeta& m, const RowRegs& Q, int32_t* rp, uint8_t* sid) {
  const int nr = m.r1 - m.r0;
  const int a0 = m.k0 & ~3;
  const int t = threadIdx.x;
  if (t <= nr) rp[t] = Q.rp[0] - a0;
  if (t + kThreads <= nr) rp[t + kThreads] = Q.rp[1] - a0;
  if (t == 0 && 2 * kThreads <= nr) rp[2 * kThreads] = Q.rp[2] - a0;
  if (t < nr) sid[t] = Q.sid[0];
  if (t + kThreads < nr) sid[t + kThreads] = Q.sid[1];
}

// Products D_ij * x_t^(q)_j of the block's nonzeros into LDS, written as
// whole 4-element vectors at their offset from the block's aligned start.
// Entries outside [k0, k1) (neighbouring rows or the zeroed tail, all valid
// column indices) are computed too and never read.
template <int NT>
__device__ __forceinline__ void fwd_products(const BlockMeta& m, const VecRegs& R, const float* xs, int nbp,
                                             float* prod) {
  const int a0 = m.k0 & ~3;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int off = 4 * (threadIdx.x + j * kThreads);
    if (a0 + off < m.k1) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const float* xq = xs + q * nbp;
        float4 p;
        p.x = R.v[j].x * xq[R.c[j].x];
        p.y = R.v[j].y * xq[R.c[j].y];
        p.z = R.v[j].z * xq[R.c[j].z];
        p.w = R.v[j].w * xq[R.c[j].w];
        *reinterpret_cast<float4*>(prod + q * kFwdNnzMax + off) = p;
      }
    }
  }
}

// Stage the inputs of a forward pass in LDS: the penalty table, the gradient
// (completing shared adjoint columns from their pieces) and the NT trial
// vectors x_t^(q) = max(0, x_k - lambda_q g_k), or x itself for a direct
// pass.  The lead workgroup also stores the trials and their step norms.
// Ends with a workgroup barrier.
template <int NT>
__device__ __forceinline__ void stage_inputs(const FwdArgs& a, bool direct, bool lead, const float* xk,
                                             const double (&lam)[NT], float* const (&xout)[NT],
                                             PenaltyDev* tab, float* xs, float* gs, double* red,
                                             bool want_sid) {
  const int tid = threadIdx.x;
  const int nb = a.nb;
  const int nbp = pad4(nb);
  if (want_sid) {
    const double* src = reinterpret_cast<const double*>(a.pen.table);
    double* dst = reinterpret_cast<double*>(tab);
    for (int i = tid; i < 4 * a.nstruct; i += kThreads) dst[i] = src[i];
  }
  constexpr int kU = 8;   // vector entries loaded per thread per round
  if (!direct) {
    // gradient of x_k; columns shared by several adjoint workgroups are
    // completed from their pieces in workgroup order
    for (int i0 = tid; i0 < nb; i0 += kU * kThreads) {
      float v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = i0 + u * kThreads;
        v[u] = a.g[i < nb ? i : 0];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = i0 + u * kThreads;
        if (i < nb) gs[i] = v[u];
      }
    }
    if (a.shared_cols != nullptr) {
      __syncthreads();
      for (int e = tid; e < a.nshared; e += kThreads) {
        const int4 sc = a.shared_cols[e];
        double tot = a.pieces[2 * sc.y + 1];
        for (int w = sc.y + 1; w < sc.z; ++w) tot += a.pieces[2 * w];
        tot += a.pieces[2 * sc.z];
        gs[sc.x] = static_cast<float>(a.g_scale * tot);
      }
    }
    __syncthreads();
  }
  double sq[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) sq[q] = 0.0;
  for (int i0 = tid; i0 < nb; i0 += kU * kThreads) {
    float xv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kThreads;
      xv[u] = xk[i < nb ? i : 0];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kThreads;
      if (i < nb) {
        if (direct) {
#pragma unroll
          for (int q = 0; q < NT; ++q) xs[q * nbp + i] = xv[u];
        } else {
          const float gi = gs[i];
#pragma unroll
          for (int q = 0; q < NT; ++q) {
            const float t = trial_point(xv[u], gi, lam[q]);
            xs[q * nbp + i] = t;
            if (lead) {
              xout[q][i] = t;
              const double dl = static_cast<double>(t) - static_cast<double>(xv[u]);
              sq[q] += dl * dl;
            }
          }
        }
      }
    }
  }
  if (lead) {
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const double t = block_sum(sq[q], red);
      if (tid == 0) a.partials[NT * gridDim.x + q] = t;
    }
  }
  __syncthreads();

}

// Forward pass.  Each workgroup stages the NT trial vectors
// x_t^(q) = max(0, x_k - lambda_q g_k) and the penalty table in LDS
// (workgroup 0 also stores the trials and their step norms), then walks its
// contiguous range of row blocks (at most kFwdPartNnz nonzeros each).  The
// next block's col_idx/val (16-byte loads), row pointers and structure ids are
// in flight while the current block's rows are summed from LDS by
// lanes-per-row groups and the penalty epilogue writes r and accumulates G.
template <int NT>
__global__ __launch_bounds__(kThreads) void fwd_kernel(FwdArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nb = a.nb;
  const int nbp = pad4(nb);
  PenaltyDev* tab = reinterpret_cast<PenaltyDev*>(smem);
  float* xs = reinterpret_cast<float*>(tab + a.nstruct);
  float* gs = xs + NT * nbp;
  float* prod = gs + nbp;
  int32_t* rp = reinterpret_cast<int32_t*>(prod + NT * kFwdNnzMax);
  uint8_t* sidl = reinterpret_cast<uint8_t*>(rp + kFwdRowsMax + 1);
  __shared__ double red[kWaves];
  __shared__ float redf[kWaves];

  const int tid = threadIdx.x;
  const bool solve = (a.mode == FWD_SOLVE);
  const bool want_sid = (a.mode != FWD_PLAIN);
  int ntr = 1;
  bool direct = true;
  double lam[NT];
  float* rout[NT];
  float* xout[NT];
  const float* xk = a.x;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    lam[q] = 0.0;
    rout[q] = nullptr;
    xout[q] = nullptr;
  }
  if (solve) {
    const SolverState* st = a.st_in;
    // the state passes through unchanged (word copy by workgroup 0)
    constexpr int kWords = static_cast<int>(sizeof(SolverState) / sizeof(int32_t));
    if (blockIdx.x == 0 && tid < kWords)
      reinterpret_cast<int32_t*>(a.st_out)[tid] = reinterpret_cast<const int32_t*>(st)[tid];
    const int phase = st->phase;
    if (phase == PH_DONE) return;
    direct = (phase == PH_INIT);
    ntr = direct ? 1 : NT;
    const int xi = st->xi, acc = st->acc;
    xk = select_buf(a.xbuf, xi);
    lam[0] = st->lambda;
    const double alpha = st->alpha;
#pragma unroll
    for (int q = 1; q < NT; ++q) lam[q] = lam[q - 1] / alpha;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      rout[q] = select_buf(a.rbuf, (acc + 1 + q) % (NT + 1));
      xout[q] = select_buf(a.xbuf, (xi + 1 + q) % (NT + 1));
    }
  }

  int b0, b1;
  work_range(a.nblocks, b0, b1);
  // first block's data in flight while the trial vectors are staged
  VecRegs R;
  RowRegs Q;
  BlockMeta cur{0, 0, 0, 0}, nxt{0, 0, 0, 0};
  if (b0 < b1) {
    cur = block_meta(a, b0);
    if (cur.k1 - cur.k0 <= kFwdPartNnz) {
      issue_vec(a.col_idx, a.val, cur.k0 & ~3, cur.k1, R);
      issue_rows(a, cur, want_sid, Q);
    }
    if (b0 + 1 < b1) nxt = block_meta(a, b0 + 1);
  }

  stage_inputs<NT>(a, direct, solve && !direct && blockIdx.x == 0, xk, lam, xout, tab, xs, gs, red, want_sid);

  double pacc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) pacc[q] = 0.0;

  for (int b = b0; b < b1; ++b) {
    const bool more = (b + 1 < b1);
    if (cur.k1 - cur.k0 > kFwdPartNnz) {
      // a single row longer than an LDS block: all lanes stride over it
      float s[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) s[q] = 0.f;
      for (int k = cur.k0 + tid; k < cur.k1; k += kThreads) {
        const int c = a.col_idx[k];
        const float v = a.val[k];
#pragma unroll
        for (int q = 0; q < NT; ++q) s[q] = fmaf(v, xs[q * nbp + c], s[q]);
      }
#pragma unroll
      for (int q = 0; q < NT; ++q) s[q] = block_sum(s[q], redf);
      if (tid == 0) row_epilogue<NT>(a, cur.r0, want_sid ? a.pen.sid[cur.r0] : 0, tab, s, pacc, rout, ntr);
      if (more) {
        cur = nxt;
        if (cur.k1 - cur.k0 <= kFwdPartNnz) {
          issue_vec(a.col_idx, a.val, cur.k0 & ~3, cur.k1, R);
          issue_rows(a, cur, want_sid, Q);
        }
        if (b + 2 < b1) nxt = block_meta(a, b + 2);
      }
      continue;
    }
    const int nr = cur.r1 - cur.r0;
    fwd_products<NT>(cur, R, xs, nbp, prod);
    stage_rows(cur, Q, rp, sidl);
    __syncthreads();
    const BlockMeta blk = cur;
    if (more) {
      cur = nxt;
      if (cur.k1 - cur.k0 <= kFwdPartNnz) {
        issue_vec(a.col_idx, a.val, cur.k0 & ~3, cur.k1, R);
        issue_rows(a, cur, want_sid, Q);
      }
      if (b + 2 < b1) nxt = block_meta(a, b + 2);
    }
    const int L = lanes_per_row(nr);
    const int lane = tid & (L - 1);
    for (int row = tid / L; row < nr; row += kThreads / L) {
      const int s0 = rp[row], s1 = rp[row + 1];
      float s[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) s[q] = 0.f;
      // four independent LDS reads per round; slots past the row read as 0
      for (int k = s0 + lane; k < s1; k += 4 * L) {
#pragma unroll
        for (int q = 0; q < NT; ++q) {
          const float* pq = prod + q * kFwdNnzMax;
          float v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kk = k + u * L;
            const float t = pq[kk < kFwdNnzMax ? kk : kFwdNnzMax - 1];
            v[u] = (kk < s1) ? t : 0.0f;
          }
          s[q] += (v[0] + v[1]) + (v[2] + v[3]);
        }
      }
      for (int off = L >> 1; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < NT; ++q) s[q] += __shfl_xor(s[q], off, 64);
      }
      if (lane == 0) row_epilogue<NT>(a, blk.r0 + row, sidl[row], tab, s, pacc, rout, ntr);
    }
    __syncthreads();
  }

#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const double t = block_sum(pacc[q], red);
    if (tid == 0) a.partials[q * gridDim.x + blockIdx.x] = t;
  }
}

// ---- wave-granular forward pass --------------------------------------------------
// Same computation as fwd_kernel, but each of the four waves of a workgroup
// streams its own range of small row blocks (at most kWavePartNnz nonzeros):
// the products, row pointers and structure ids of a block live in the wave's
// own LDS region, so blocks need no workgroup barrier, and sixteen or more
// independent streams per compute unit keep memory busy.
struct WaveRows {
  int rp[5];
  uint8_t sid[4];
};

__device__ __forceinline__ void wave_issue(const FwdArgs& a, const BlockMeta& m, bool want_sid, int lane,
                                           VecRegs& R, WaveRows& Q) {
  const int a0 = m.k0 & ~3;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    int e0 = a0 + 4 * (lane + 64 * j);
    e0 = (e0 < m.k1) ? e0 : 0;
    R.c[j] = *reinterpret_cast<const int4*>(a.col_idx + e0);
    R.v[j] = *reinterpret_cast<const float4*>(a.val + e0);
  }
  const int nr = m.r1 - m.r0;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const int i = lane + 64 * j;
    Q.rp[j] = a.row_ptr[m.r0 + ((i <= nr) ? i : 0)];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = lane + 64 * j;
    Q.sid[j] = want_sid ? a.pen.sid[m.r0 + ((i < nr) ? i : 0)] : 0;
  }
}

template <int NT>
__global__ __launch_bounds__(kThreads) void fwd_wave_kernel(FwdArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nb = a.nb;
  const int nbp = pad4(nb);
  PenaltyDev* tab = reinterpret_cast<PenaltyDev*>(smem);
  float* xs = reinterpret_cast<float*>(tab + a.nstruct);
  float* gs = xs + NT * nbp;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int kWaveBytes = ((NT * kWaveNnz + kWaveRowsMax + 1) * 4 + kWaveRowsMax + 15) & ~15;
  unsigned char* wbase = reinterpret_cast<unsigned char*>(gs + nbp) + wv * kWaveBytes;
  float* prod = reinterpret_cast<float*>(wbase);
  int32_t* rp = reinterpret_cast<int32_t*>(prod + NT * kWaveNnz);
  uint8_t* sidl = reinterpret_cast<uint8_t*>(rp + kWaveRowsMax + 1);
  __shared__ double red[kWaves];

  const int tid = threadIdx.x;
  const bool solve = (a.mode == FWD_SOLVE);
  const bool want_sid = (a.mode != FWD_PLAIN);
  int ntr = 1;
  bool direct = true;
  double lam[NT];
  float* rout[NT];
  float* xout[NT];
  const float* xk = a.x;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    lam[q] = 0.0;
    rout[q] = nullptr;
    xout[q] = nullptr;
  }
  if (solve) {
    const SolverState* st = a.st_in;
    constexpr int kWords = static_cast<int>(sizeof(SolverState) / sizeof(int32_t));
    if (blockIdx.x == 0 && tid < kWords)
      reinterpret_cast<int32_t*>(a.st_out)[tid] = reinterpret_cast<const int32_t*>(st)[tid];
    const int phase = st->phase;
    if (phase == PH_DONE) return;
    direct = (phase == PH_INIT);
    ntr = direct ? 1 : NT;
    const int xi = st->xi, acc = st->acc;
    xk = select_buf(a.xbuf, xi);
    lam[0] = st->lambda;
    const double alpha = st->alpha;
#pragma unroll
    for (int q = 1; q < NT; ++q) lam[q] = lam[q - 1] / alpha;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      rout[q] = select_buf(a.rbuf, (acc + 1 + q) % (NT + 1));
      xout[q] = select_buf(a.xbuf, (xi + 1 + q) % (NT + 1));
    }
  }

  // this wave's contiguous range of row blocks
  const int G = gridDim.x, w = blockIdx.x;
  const int lw = (G % kXcds == 0) ? (w % kXcds) * (G / kXcds) + w / kXcds : w;
  const long long W = static_cast<long long>(G) * kWaves, gw = static_cast<long long>(lw) * kWaves + wv;
  const int b0 = static_cast<int>(gw * a.nwblocks / W), b1 = static_cast<int>((gw + 1) * a.nwblocks / W);
  auto meta = [&](int b) {
    BlockMeta m;
    m.r0 = a.wblock_row[b];
    m.r1 = a.wblock_row[b + 1];
    m.k0 = a.wblock_k0[b];
    m.k1 = a.wblock_k0[b + 1];
    return m;
  };
  VecRegs R;
  WaveRows Q;
  BlockMeta cur{0, 0, 0, 0}, nxt{0, 0, 0, 0};
  if (b0 < b1) {
    cur = meta(b0);
    if (cur.k1 - cur.k0 <= kWavePartNnz) wave_issue(a, cur, want_sid, lane, R, Q);
    if (b0 + 1 < b1) nxt = meta(b0 + 1);
  }

  stage_inputs<NT>(a, direct, solve && !direct && blockIdx.x == 0, xk, lam, xout, tab, xs, gs, red, want_sid);

  double pacc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) pacc[q] = 0.0;

  for (int b = b0; b < b1; ++b) {
    const bool more = (b + 1 < b1);
    if (cur.k1 - cur.k0 > kWavePartNnz) {
      // a single row longer than a wave block: the wave strides over it
      float s[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) s[q] = 0.f;
      for (int k = cur.k0 + lane; k < cur.k1; k += 64) {
        const int c = a.col_idx[k];
        const float v = a.val[k];
#pragma unroll
        for (int q = 0; q < NT; ++q) s[q] = fmaf(v, xs[q * nbp + c], s[q]);
      }
#pragma unroll
      for (int q = 0; q < NT; ++q) s[q] = wave_sum(s[q]);
      if (lane == 0) row_epilogue<NT>(a, cur.r0, want_sid ? a.pen.sid[cur.r0] : 0, tab, s, pacc, rout, ntr);
      if (more) {
        cur = nxt;
        if (cur.k1 - cur.k0 <= kWavePartNnz) wave_issue(a, cur, want_sid, lane, R, Q);
        if (b + 2 < b1) nxt = meta(b + 2);
      }
      continue;
    }
    const int a0 = cur.k0 & ~3;
    const int nr = cur.r1 - cur.r0;
    // products and row data of this block into the wave's LDS region
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int off = 4 * (lane + 64 * j);
      if (a0 + off < cur.k1) {
#pragma unroll
        for (int q = 0; q < NT; ++q) {
          const float* xq = xs + q * nbp;
          float4 p;
          p.x = R.v[j].x * xq[R.c[j].x];
          p.y = R.v[j].y * xq[R.c[j].y];
          p.z = R.v[j].z * xq[R.c[j].z];
          p.w = R.v[j].w * xq[R.c[j].w];
          *reinterpret_cast<float4*>(prod + q * kWaveNnz + off) = p;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int i = lane + 64 * j;
      if (i <= nr) rp[i] = Q.rp[j] - a0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = lane + 64 * j;
      if (i < nr) sidl[i] = Q.sid[j];
    }
    // LDS operations of one wave complete in order; the fence only keeps the
    // compiler from moving the reads above the writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const BlockMeta blk = cur;
    if (more) {
      cur = nxt;
      if (cur.k1 - cur.k0 <= kWavePartNnz) wave_issue(a, cur, want_sid, lane, R, Q);
      if (b + 2 < b1) nxt = meta(b + 2);
    }
    int L = 64;
    while (L > 1 && L * nr > 64) L >>= 1;
    const int sub = lane & (L - 1);
    for (int row = lane / L; row < nr; row += 64 / L) {
      const int s0 = rp[row], s1 = rp[row + 1];
      float s[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) s[q] = 0.f;
      for (int k = s0 + sub; k < s1; k += 4 * L) {
#pragma unroll
        for (int q = 0; q < NT; ++q) {
          const float* pq = prod + q * kWaveNnz;
          float v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kk = k + u * L;
            const float t = pq[kk < kWaveNnz ? kk : kWaveNnz - 1];
            v[u] = (kk < s1) ? t : 0.0f;
          }
          s[q] += (v[0] + v[1]) + (v[2] + v[3]);
        }
      }
      for (int off = L >> 1; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < NT; ++q) s[q] += __shfl_xor(s[q], off, 64);
      }
      if (sub == 0) row_epilogue<NT>(a, blk.r0 + row, sidl[row], tab, s, pacc, rout, ntr);
    }
    // the next block's LDS writes must not overtake this block's reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }

#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const double t = block_sum(pacc[q], red);
    if (tid == 0) a.partials[q * gridDim.x + blockIdx.x] = t;
  }
}

// ---- adjoint pass ----------------------------------------------------------------
// Residual gathers for the nonzeros of R: all eight are issued together
// (every index held in R is a valid row: a real entry or the zeroed tail).
struct GatherRegs {
  float r[8];
};

__device__ __forceinline__ void adj_gather(const VecRegs& R, const float* r, GatherRegs& Gr) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    Gr.r[4 * j + 0] = r[R.c[j].x];
    Gr.r[4 * j + 1] = r[R.c[j].y];
    Gr.r[4 * j + 2] = r[R.c[j].z];
    Gr.r[4 * j + 3] = r[R.c[j].w];
  }
}

// Fixed-order float64 sum of val * r over this thread's nonzeros of the
// round starting at `base`, counting only [k0, k1).
__device__ __forceinline__ double adj_accumulate(const VecRegs& R, const GatherRegs& Gr, int base, int k0,
                                                 int k1) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int e0 = base + 4 * (threadIdx.x + j * kThreads);
    const float vv[4] = {R.v[j].x, R.v[j].y, R.v[j].z, R.v[j].w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool in = (e0 + i >= k0) && (e0 + i < k1);
      s += static_cast<double>(in ? vv[i] : 0.0f) * static_cast<double>(Gr.r[4 * j + i]);
    }
  }
  return s;
}

__device__ __forceinline__ int logical_wg() {
  const int G = gridDim.x, w = blockIdx.x;
  return (G % kXcds == 0) ? (w % kXcds) * (G / kXcds) + w / kXcds : w;
}

// Adjoint pass: in a solve, first the decision on the preceding forward pass
// (every workgroup identically; workgroup 0 stores the new state and trace
// entry), then g = scale * D^T r over this workgroup's share of the nonzeros.
template <int NT>
__global__ __launch_bounds__(kThreads) void adj_kernel(AdjArgs a) {
  __shared__ double red[kWaves];
  __shared__ Decision dec;
  const int tid = threadIdx.x;
  const int lw = logical_wg();
  const int64_t k0w = static_cast<int64_t>(lw) * a.nnz / a.grid;
  const int64_t k1w = static_cast<int64_t>(lw + 1) * a.nnz / a.grid;
  const int c0 = a.wg_c0[lw], c1 = a.wg_c1[lw];
  // the first column's first loads do not depend on the decision
  VecRegs cur, nxt;
  int s0 = 0, s1 = 0;
  if (c0 < c1) {
    s0 = static_cast<int>(max(k0w, static_cast<int64_t>(a.col_ptr[c0])));
    s1 = static_cast<int>(min(k1w, static_cast<int64_t>(a.col_ptr[c0 + 1])));
    issue_vec(a.row_idx, a.val, s0 & ~3, s1, cur);
  }
  const float* r = a.r;
  if (a.solve) {
    decide<NT>(a.st_in, a.fwd_partials, a.fwd_parts, dec, red);
    if (blockIdx.x == 0 && tid == 0) {
      *a.st_out = dec.st;
      if (dec.accepted >= 0 && a.trace != nullptr && dec.st.k - 1 < dec.st.trace_cap) {
        TraceDev e;
        e.k = dec.st.k;
        e.backtracks = dec.backtracks;
        e.lambda = dec.lam;
        e.step_sq = dec.step_sq;
        e.G = dec.st.G;
        a.trace[dec.st.k - 1] = e;
      }
    }
    if (dec.st.phase != PH_NEED_GRAD) return;
    r = select_buf(a.rbuf, dec.st.acc);
  }
  constexpr int kStep = 8 * kThreads;   // nonzeros covered by one round of loads
  for (int c = c0; c < c1; ++c) {
    if (c > c0) {
      s0 = static_cast<int>(max(k0w, static_cast<int64_t>(a.col_ptr[c])));
      s1 = static_cast<int>(min(k1w, static_cast<int64_t>(a.col_ptr[c + 1])));
      issue_vec(a.row_idx, a.val, s0 & ~3, s1, cur);
    }
    double s = 0.0;
    for (int base = s0 & ~3; base < s1; base += kStep) {
      // gathers of this round first, then the next round's loads, so that
      // waiting for the gathers does not wait for the prefetch
      GatherRegs Gr;
      adj_gather(cur, r, Gr);
      issue_vec(a.row_idx, a.val, base + kStep, s1, nxt);   // past the end: first vector only
      s += adj_accumulate(cur, Gr, base, s0, s1);
      cur = nxt;
    }
    s = block_sum(s, red);
    if (tid == 0) {
      const int wlo = a.col_wlo[c], whi = a.col_whi[c];
      if (wlo == whi) {
        a.out[c] = static_cast<float>(a.scale * s);
      } else {
        if (c == c0) a.pieces[2 * lw] = s;
        if (c == c1 - 1) a.pieces[2 * lw + 1] = s;
      }
    }
  }
}

// Columns shared by several adjoint workgroups (completion not folded): the
// fixed-order sum of their pieces.  Runs after adj_kernel; in a solve only
// when that pass computed a gradient (state after the decision in `st`).
__global__ __launch_bounds__(kThreads) void adj_final_kernel(AdjArgs a, const SolverState* st) {
  if (st != nullptr && st->phase != PH_NEED_GRAD) return;
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= a.nb) return;
  const int wlo = a.col_wlo[c], whi = a.col_whi[c];
  if (wlo == whi) return;
  double tot = a.pieces[2 * wlo + 1];
  for (int w = wlo + 1; w < whi; ++w) tot += a.pieces[2 * w];
  tot += a.pieces[2 * whi];
  a.out[c] = static_cast<float>(a.scale * tot);
}

// ---- small utility kernels ----------------------------------------------------------
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

// Drop an error left behind by an unrelated earlier runtime call on this
// thread, so that check_launch reports only the launch that follows.
void clear_stale_error() { (void)hipGetLastError(); }

int grid_for(int items, int cap) {
  if (items <= 0) return 1;
  if (items <= cap) return items;
  return cap;
}

}  // namespace

size_t forward_lds_bytes(int nb, int ntrials, int nstruct, bool wave) {
  const size_t nbp = static_cast<size_t>(pad4(nb));
  size_t bytes = static_cast<size_t>(nstruct) * sizeof(PenaltyDev) +
                 (static_cast<size_t>(ntrials) * nbp + nbp) * sizeof(float);
  if (wave) {
    const size_t per_wave = ((static_cast<size_t>(ntrials) * kWaveNnz + kWaveRowsMax + 1) * 4 + kWaveRowsMax + 15) &
                            ~static_cast<size_t>(15);
    bytes += kWaves * per_wave;
  } else {
    bytes += static_cast<size_t>(ntrials) * kFwdNnzMax * sizeof(float) +
             static_cast<size_t>(kFwdRowsMax + 1) * sizeof(int32_t) + kFwdRowsMax;
  }
  return bytes;
}

int forward_grid(const imrt_ctx* ctx, const imrt_dose* D) {
  const int items = ctx->tune.fwd_wave ? (D->nwblocks + kWaves - 1) / kWaves : D->nblocks;
  return grid_for(items, ctx->tune.fwd_grid_per_cu * ctx->num_cu);
}

int adjoint_grid_for(const imrt_ctx* ctx, int64_t nnz) {
  const int64_t cap = static_cast<int64_t>(ctx->tune.adj_grid_per_cu) * ctx->num_cu;
  // at least adj_min_nnz nonzeros per workgroup, at least one workgroup
  const int64_t per = ctx->tune.adj_min_nnz;
  const int64_t want = (nnz + per - 1) / per;
  return static_cast<int>(std::max<int64_t>(1, std::min(cap, want)));
}

int launch_forward(const imrt_ctx* ctx, const imrt_dose* D, const FwdArgs& a, int ntrials, int grid,
                   hipEvent_t before, hipEvent_t after) {
  (void)D;
  clear_stale_error();
  const bool wave = ctx->tune.fwd_wave != 0;
  const size_t lds = forward_lds_bytes(a.nb, ntrials, a.nstruct, wave);
  if (lds > ctx->max_lds)
    return set_error(IMRT_EUNSUPPORTED, "forward pass: nb * trials exceeds the LDS budget");
  if (before && hipEventRecord(before, ctx->stream) != hipSuccess) return check_launch("hipEventRecord");
  if (wave) {
    switch (ntrials) {
      case 1: hipLaunchKernelGGL(fwd_wave_kernel<1>, dim3(grid), dim3(kThreads), lds, ctx->stream, a); break;
      case 2: hipLaunchKernelGGL(fwd_wave_kernel<2>, dim3(grid), dim3(kThreads), lds, ctx->stream, a); break;
      case 4: hipLaunchKernelGGL(fwd_wave_kernel<4>, dim3(grid), dim3(kThreads), lds, ctx->stream, a); break;
      default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
    }
  } else {
    switch (ntrials) {
      case 1: hipLaunchKernelGGL(fwd_kernel<1>, dim3(grid), dim3(kThreads), lds, ctx->stream, a); break;
      case 2: hipLaunchKernelGGL(fwd_kernel<2>, dim3(grid), dim3(kThreads), lds, ctx->stream, a); break;
      case 4: hipLaunchKernelGGL(fwd_kernel<4>, dim3(grid), dim3(kThreads), lds, ctx->stream, a); break;
      default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
    }
  }
  const int rc = check_launch("fwd_kernel");
  if (rc == IMRT_OK && after && hipEventRecord(after, ctx->stream) != hipSuccess) return check_launch("hipEventRecord");
  return rc;
}

int launch_adjoint(const imrt_ctx* ctx, const imrt_dose* D, const AdjArgs& a, int ntrials, hipEvent_t before,
                   hipEvent_t after) {
  clear_stale_error();
  if (before && hipEventRecord(before, ctx->stream) != hipSuccess) return check_launch("hipEventRecord");
  switch (ntrials) {
    case 1: hipLaunchKernelGGL(adj_kernel<1>, dim3(a.grid), dim3(kThreads), 0, ctx->stream, a); break;
    case 2: hipLaunchKernelGGL(adj_kernel<2>, dim3(a.grid), dim3(kThreads), 0, ctx->stream, a); break;
    case 4: hipLaunchKernelGGL(adj_kernel<4>, dim3(a.grid), dim3(kThreads), 0, ctx->stream, a); break;
    default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
  }
  int rc = check_launch("adj_kernel");
  if (rc) return rc;
  if (after && hipEventRecord(after, ctx->stream) != hipSuccess) return check_launch("hipEventRecord");
  if (!a.fold) {
    const int g2 = (a.nb + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(adj_final_kernel, dim3(g2), dim3(kThreads), 0, ctx->stream, a,
                       a.solve ? static_cast<const SolverState*>(a.st_out) : nullptr);
    rc = check_launch("adj_final_kernel");
  }
  (void)D;
  return rc;
}

int launch_sum(const imrt_ctx* ctx, const double* parts, int n, double* out) {
  clear_stale_error();
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kThreads), 0, ctx->stream, parts, n, out);
  return check_launch("sum_kernel");
}

int launch_project(const imrt_ctx* ctx, const float* x, const float* g, double lambda, int nb,
                   float* x_out, double* s_out) {
  clear_stale_error();
  hipLaunchKernelGGL(project_kernel, dim3(1), dim3(kThreads), 0, ctx->stream, x, g, lambda, nb, x_out, s_out);
  return check_launch("project_kernel");
}

int launch_normalize(const imrt_ctx* ctx, const float* w, int nb, float* v_out, double* norm_out) {
  clear_stale_error();
  hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(kThreads), 0, ctx->stream, w, nb, v_out, norm_out);
  return check_launch("normalize_kernel");
}

}  // namespace imrt
