// Hot-path kernels of the gradient-projection / Armijo solver for gfx950.
//
//  fwd_kernel / fwd_wave_kernel
//               trial points x_t = max(0, x_k - lambda g) (steps 2 and 4)
//               staged in LDS, forward dose z = D x over CSR (Section 2.1),
//               penalty residual and objective partials (Eqs. (1)-(2)), in
//               one pass over D.
//  adj_kernel   line-search decision on the preceding forward pass (Armijo
//               test of Eq. (5), stopping test of step 5), taken identically
//               by every workgroup, then the beamlet-parallel adjoint
//               g = 2 D^T r over CSC for an accepted, unfinished iterate.
//  adj_final    completes shared columns outside a solve (in a solve the
//               next forward pass completes them while staging its trials).
//
// The solver state is double-buffered: a pass reads one copy and workgroup 0
// writes the other, so no workgroup ever sees a state written during its own
// pass.  Every reduction runs in a fixed order, so results are
// bit-reproducible and independent of workgroup timing; there are no
// floating-point atomics.  (The waves of a wave-granular forward workgroup
// take row blocks from an integer counter in LDS, but a block's rows and its
// objective contribution come out the same whichever wave takes it, and the
// contributions are added in block order.)  Work is dealt to workgroups in contiguous ranges,
// consecutive ranges on the same accelerator die (workgroups are dispatched
// round-robin over the 8 dies), so neighbouring beamlet columns share that
// die's L2 for their residual gathers.
#include <algorithm>
#include <cstddef>
#include <type_traits>
#include <cmath>

#include <hip/hip_ext.h>

#include "imrt_internal.h"

namespace imrt {
namespace {

// A workgroup's place in its pass: index w among the pass's G workgroups.  A
// single plan's pass has one workgroup per dispatch slot; a batched pass
// runs several plans' passes in one dispatch, each workgroup looking up its
// plan and its slot in that plan's pass, so every plan computes exactly what
// it computes alone.
struct Slot {
  int w, G;
};

// Trial point of steps 2/4: max(0, x - lambda g), evaluated in float64 and
// rounded once to float32.  NaN propagates (it is not clipped to zero).
__device__ __forceinline__ float trial_point(float x, float g, double lam) {
#pragma clang fp contract(off)
  const double t = static_cast<double>(x) - lam * static_cast<double>(g);
  return static_cast<float>(t < 0.0 ? 0.0 : t);
}

// ---- cross-lane sums ----------------------------------------------------------
// Data-parallel-primitive (DPP) moves within a wave: swaps inside quads, the
// mirrors of 8- and 16-lane rows, and the row broadcasts of lanes 15 and 31.
// Lanes a row mask leaves out receive 0.  The order of every sum is fixed.
constexpr int kDppQuadXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xF, false));
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
  const int2 w = __builtin_bit_cast(int2, v);
  int2 o;
  o.x = __builtin_amdgcn_update_dpp(0, w.x, CTRL, ROWS, 0xF, false);
  o.y = __builtin_amdgcn_update_dpp(0, w.y, CTRL, ROWS, 0xF, false);
  return __builtin_bit_cast(double, o);
}

// Sum over each aligned group of L lanes; valid in the group's last lane
// (lane % L == L - 1).
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
  if constexpr (L >= 2) v += dpp_move<kDppQuadXor1, 0xF>(v);
  if constexpr (L >= 4) v += dpp_move<kDppQuadXor2, 0xF>(v);
  if constexpr (L >= 8) v += dpp_move<kDppRowHalfMirror, 0xF>(v);
  if constexpr (L >= 16) v += dpp_move<kDppRowMirror, 0xF>(v);
  if constexpr (L >= 32) v += dpp_move<kDppRowBcast15, 0xA>(v);
  if constexpr (L >= 64) v += dpp_move<kDppRowBcast31, 0xC>(v);
  return v;
}

// Sum over the wave; valid in lane 63.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  return group_sum<64>(v);
}

// Sum of v over a workgroup of WAVES waves in a fixed order; the result is
// valid in thread 0.
template <typename T, int WAVES = kWaves>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) sh[w] = v;
  __syncthreads();
  T t = T(0);
  if (threadIdx.x == 0) {
    t = sh[0];
#pragma unroll
    for (int i = 1; i < WAVES; ++i) t += sh[i];
  }
  __syncthreads();
  return t;
}

// ---- buffer resources -----------------------------------------------------------
// A raw buffer descriptor built from a wave-uniform base address and length:
// loads take 32-bit offsets, and a lane whose offset lies past the length
// reads zeros without touching memory.  Lengths are kept multiples of the
// access size, so an access is either wholly inside or wholly outside.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;   // CDNA descriptor word 3: 32-bit data, no swizzle

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, static_cast<int>(bytes), kRsrcWord3);
}
__device__ __forceinline__ int4 load_i4(rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(int4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ int load_i32(rsrc_t r, uint32_t off) {
  return static_cast<int>(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ float load_f32(rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double load_f64(rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ uint32_t load_u8(rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
}
// Loads of the matrix streams with cache policy CP: 0 the default, 2 the
// non-temporal policy, for matrices larger than the last-level cache (a
// pass's stream would otherwise evict the vectors and tables the passes
// reuse; the values read are the same either way).
template <int CP>
__device__ __forceinline__ int4 load_i4s(rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(int4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CP));
}
template <int CP>
__device__ __forceinline__ float4 load_f4s(rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CP));
}
template <int CP>
__device__ __forceinline__ uint2 load_u2s(rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, CP));
}
__device__ __forceinline__ void store_f32(rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

// Everything the decision reads is loaded by decide_start: the first round of
// partials (four per thread and trial), the state (one 32-bit word per lane
// of every wave) and the first step-norm part of every trial.
// The loads are not combined with anything here, so that the compiler waits
// for them only where decide uses them, after the caller's later loads were
// issued.
constexpr int kStateWords = static_cast<int>(sizeof(SolverState) / sizeof(int32_t));
static_assert(kStateWords <= 64, "the state is loaded one word per lane of a wave");

// floor(i * n / parts) for wave-uniform arguments (64-bit product).
__device__ __forceinline__ int split_point(int i, int n, int parts) {
  return uniform(static_cast<int>(static_cast<long long>(i) * n / parts));
}

// Fields of a state loaded one 32-bit word per lane (lane i holds word i).
__device__ __forceinline__ int state_int(int32_t sw, size_t byte_off) {
  return __builtin_amdgcn_readlane(sw, static_cast<int>(byte_off / 4));
}
__device__ __forceinline__ double state_f64(int32_t sw, size_t byte_off) {
  const int lo = __builtin_amdgcn_readlane(sw, static_cast<int>(byte_off / 4));
  const int hi = __builtin_amdgcn_readlane(sw, static_cast<int>(byte_off / 4) + 1);
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<uint32_t>(hi)) << 32) |
                                        static_cast<uint32_t>(lo));
}

template <int NT>
struct DecideLoads {
  double v[NT][4];
  double step0[NT];
  int32_t sw;
};

template <int NT>
__device__ __forceinline__ void decide_start(const AdjArgs& a, DecideLoads<NT>& L) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int nparts = a.fwd_parts, nsteps = a.step_parts;
  const rsrc_t rp = make_rsrc(a.fwd_partials, 8u * NT * static_cast<uint32_t>(nparts));
  const rsrc_t rs = make_rsrc(a.step_partials, 8u * NT * static_cast<uint32_t>(nsteps));
  const rsrc_t rst = make_rsrc(a.st_in, static_cast<uint32_t>(sizeof(SolverState)));
#pragma unroll
  for (int q = 0; q < NT; ++q) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = tid + u * kThreads;
      L.v[q][u] = load_f64(rp, 8u * static_cast<uint32_t>(q * nparts + (i < nparts ? i : 0)));
    }
    L.step0[q] = load_f64(rs, 8u * static_cast<uint32_t>(q * nsteps));
  }
  L.sw = load_i32(rst, 4u * static_cast<uint32_t>(lane < kStateWords ? lane : 0));
}

template <int NT>
__device__ void decide(const double* partials, int nparts, const double* steps, int nsteps,
                       const DecideLoads<NT>& L, Decision& dec, double* red, double G_add) {
#pragma clang fp contract(off)
  __shared__ double Gq[NT];
  const int tid = threadIdx.x;
  double s[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    // four values per round, summed in index order
    s[q] = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) s[q] += (tid + u * kThreads < nparts) ? L.v[q][u] : 0.0;
    const double* pq = partials + q * nparts;
    for (int i0 = tid + 4 * kThreads; i0 < nparts; i0 += 4 * kThreads) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * kThreads;
        v[u] = pq[i < nparts ? i : 0];
        v[u] = (i < nparts) ? v[u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) s[q] += v[u];
    }
  }
  if (tid < kStateWords) reinterpret_cast<int32_t*>(&dec.st)[tid] = L.sw;
  if (tid == 0) dec.accepted = -1;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const double t = block_sum(s[q], red);
    if (tid == 0) Gq[q] = t + G_add;
  }
  if (dec.st.phase == PH_DONE) return;
  const bool init = (dec.st.phase == PH_INIT);
  if (tid == 0) {
    SolverState st = dec.st;
    st.n_fwd += 1;
    if (init) {
      // (st.lambda already holds the first trial step: lambda0, or for a
      // warm-started resumed solve alpha times the step accepted last)
      const double G0 = Gq[0];
      st.G = G0;
      st.G_init = G0;
      if (!st.resume) st.G_prev = G0;
      st.acc = 0;
      st.m = 0;
      if (!isfinite(G0)) {
        st.status = IMRT_NUMERIC;
        st.phase = PH_DONE;
      } else if (st.resume && !st.fixed && (G0 == 0.0 || fabs(G0 - st.G_prev) / G0 < st.delta)) {
        st.status = IMRT_CONVERGED;   // step 5 on the pair the interrupted solve ended with
        st.phase = PH_DONE;
      } else if (st.max_iter <= 0) {
        st.status = IMRT_MAX_ITER;
        st.phase = PH_DONE;
      } else {
        st.phase = PH_NEED_GRAD;
      }
    } else {
      double sq[NT];
      for (int q = 0; q < NT; ++q) {
        double t = 0.0;
        if (nsteps > 0) t += L.step0[q];
        for (int w = 1; w < nsteps; ++w) t += steps[q * nsteps + w];
        sq[q] = t;
      }
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
        st.acc = accepted;
        st.xi = (st.xi + 1 + accepted) % (NT + 1);
        st.m = 0;
        st.lambda = st.warm ? st.alpha * l : st.lambda0;   // step 2 of the next iteration
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

// ---- stored values --------------------------------------------------------------
// A lane holds its entries in groups of four: float32 storage as int4 column
// indices and float4 values, 16-bit storage as two 32-bit words of packed
// 16-bit indices or codes (entry u in the low half of word u / 2 when u is
// even, in the high half when odd); the ST_F32C16 layout pairs packed 16-bit
// indices with float4 values.
template <int ST>
__device__ __forceinline__ float code_value(uint32_t h) {
  if constexpr (ST == ST_BF16) {
    return __uint_as_float(h << 16);
  } else {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(h)));
  }
}
__device__ __forceinline__ uint32_t half_of(const uint2& w, int u) {
  const uint32_t x = (u < 2) ? w.x : w.y;
  return (u & 1) ? (x >> 16) : (x & 0xFFFFu);
}
__device__ __forceinline__ int col_of(const int4& c, int u) {
  return u == 0 ? c.x : u == 1 ? c.y : u == 2 ? c.z : c.w;
}
__device__ __forceinline__ int col_of(const uint2& c, int u) { return static_cast<int>(half_of(c, u)); }
template <int ST>
__device__ __forceinline__ float val_of(const float4& v, int u) {
  return u == 0 ? v.x : u == 1 ? v.y : u == 2 ? v.z : v.w;
}
template <int ST>
__device__ __forceinline__ float val_of(const uint2& v, int u) {
  return code_value<ST>(half_of(v, u));
}
template <int ST>
using ColGroup = std::conditional_t<ST == ST_F32, int4, uint2>;
template <int ST>
using ValGroup = std::conditional_t<coded(ST), uint2, float4>;

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

// Staging of a forward pass's inputs in LDS: the penalty table and the NT
// vectors the pass multiplies by (row q of `src`, stride pad4(nb)).  The
// first round of loads (2048 entries per vector, and the table) goes to
// registers so that a caller can issue further loads before it waits for
// them; stage_finish stores them, stages the rest and ends with a barrier.
constexpr int kStageU = 8;   // entries per thread per round and vector

template <int NT>
struct StageRegs {
  float v[NT][kStageU];
  float sc[kStageU];
  double tab;
};

template <int NT, int THREADS = kThreads, int ST = ST_F32>
__device__ __forceinline__ void stage_start(const FwdArgs& a, const float* src, bool want_sid, StageRegs<NT>& R) {
  const int tid = threadIdx.x, nb = a.nb, nbp = pad4(nb);
  // (slots wholly past the last entry for this wave issue no loads)
  const int wave0 = uniform(tid - (tid & 63));
#pragma unroll
  for (int q = 0; q < NT; ++q) {
#pragma unroll
    for (int u = 0; u < kStageU; ++u) {
      const int i = tid + u * THREADS;
      R.v[q][u] = (wave0 + u * THREADS < nb) ? src[q * nbp + (i < nb ? i : 0)] : 0.0f;
    }
  }
  if constexpr (coded(ST)) {
#pragma unroll
    for (int u = 0; u < kStageU; ++u) {
      const int i = tid + u * THREADS;
      R.sc[u] = (wave0 + u * THREADS < nb) ? a.col_scale[i < nb ? i : 0] : 0.0f;
    }
  }
  // first THREADS doubles of the table (4 per structure); the rest in stage_finish
  R.tab = (want_sid && tid < 4 * a.nstruct) ? reinterpret_cast<const double*>(a.pen.table)[tid] : 0.0;
}

// With 16-bit storage the staged vector is scaled by the beamlet scales, so
// that the products use the codes directly: sum_i q_ji (s_i x_i).
template <int NT, int THREADS = kThreads, int ST = ST_F32>
__device__ __forceinline__ void stage_finish(const FwdArgs& a, const float* src, bool want_sid,
                                             const StageRegs<NT>& R, PenaltyDev* tab, float* xs) {
  const int tid = threadIdx.x, nb = a.nb, nbp = pad4(nb);
  if (want_sid) {
    double* dst = reinterpret_cast<double*>(tab);
    if (tid < 4 * a.nstruct) dst[tid] = R.tab;
    for (int i = tid + THREADS; i < 4 * a.nstruct; i += THREADS)
      dst[i] = reinterpret_cast<const double*>(a.pen.table)[i];
  }
#pragma unroll
  for (int q = 0; q < NT; ++q) {
#pragma unroll
    for (int u = 0; u < kStageU; ++u) {
      const int i = tid + u * THREADS;
      if (i < nb) xs[q * nbp + i] = !coded(ST) ? R.v[q][u] : R.v[q][u] * R.sc[u];
    }
  }
  for (int i0 = tid + kStageU * THREADS; i0 < nb; i0 += kStageU * THREADS) {
    float v[NT][kStageU];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
#pragma unroll
      for (int u = 0; u < kStageU; ++u) {
        const int i = i0 + u * THREADS;
        v[q][u] = src[q * nbp + (i < nb ? i : 0)];
        if constexpr (coded(ST)) v[q][u] *= a.col_scale[i < nb ? i : 0];
      }
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) {
#pragma unroll
      for (int u = 0; u < kStageU; ++u) {
        const int i = i0 + u * THREADS;
        if (i < nb) xs[q * nbp + i] = v[q][u];
      }
    }
  }
  __syncthreads();
}

// Trial staging of a solve's forward pass: for every beamlet the gradient
// entry (columns shared by two adjoint workgroups completed from their two
// float64 pieces, in order; by more, from the per-workgroup pieces), the
// iterate x_k (the state names its buffer; every candidate is loaded before
// the state arrives) and the NT trial points x_t^(q) = max(0, x_k - lambda_q g)
// (Eq. (4) with the projection of step 2), written to LDS.  The lead
// workgroup also stores the trials in their iterate buffers and reduces
// their step norms ||x_t^(q) - x_k||^2.  The initial evaluation stages x_1.
constexpr int kTrialU = 4;   // beamlets per thread per round of trial staging

template <int NT>
struct TrialRegs {
  float xc[NT + 1][kTrialU];
  float g[kTrialU];
  double p0[kTrialU], p1[kTrialU];
  uint32_t kind[kTrialU];
  float sc[kTrialU];
  double tab;
};

// Buffer loads bounded by nb: the slots of a thread past the last beamlet
// read zeros and send no request to memory.
template <int NT, int THREADS = kThreads, int ST = ST_F32>
__device__ __forceinline__ void trial_load(const FwdArgs& a, int i0, TrialRegs<NT>& R) {
  const uint32_t nb = static_cast<uint32_t>(a.nb);
  rsrc_t rx[NT + 1];
#pragma unroll
  for (int j = 0; j <= NT; ++j) rx[j] = make_rsrc(a.xbuf[j], 4u * nb);
  const rsrc_t rg = make_rsrc(a.g, 4u * nb);
  const rsrc_t rp = make_rsrc(a.pieces_col, a.pieces_col ? 16u * nb : 0u);
  const rsrc_t rk = make_rsrc(a.col_kind, nb);
  const rsrc_t rs = make_rsrc(a.col_scale, (coded(ST) && a.col_scale) ? 4u * nb : 0u);
  // a slot wholly past the last beamlet for this wave issues no loads at
  // all (out-of-range lanes cost address cycles even when they read zeros)
  const int wave0 = uniform(i0 - static_cast<int>(threadIdx.x & 63));
#pragma unroll
  for (int u = 0; u < kTrialU; ++u) {
    const uint32_t i = static_cast<uint32_t>(i0 + u * THREADS);
    if (wave0 + u * THREADS < a.nb) {
#pragma unroll
      for (int j = 0; j <= NT; ++j) R.xc[j][u] = load_f32(rx[j], 4u * i);
      R.g[u] = load_f32(rg, 4u * i);
      R.p0[u] = load_f64(rp, 16u * i);
      R.p1[u] = load_f64(rp, 16u * i + 8u);
      R.kind[u] = load_u8(rk, i);
      if constexpr (coded(ST)) R.sc[u] = load_f32(rs, 4u * i);
    } else {
#pragma unroll
      for (int j = 0; j <= NT; ++j) R.xc[j][u] = 0.0f;
      R.g[u] = 0.0f;
      R.p0[u] = R.p1[u] = 0.0;
      R.kind[u] = 0;
      R.sc[u] = 0.0f;
    }
  }
}

// Sum of the pieces of a column shared by three or more adjoint workgroups
// (16-bit storage: of the codes' products, before the beamlet scale).
__device__ __forceinline__ double pieces_sum(const FwdArgs& a, int c) {
  const int wlo = a.col_wlo[c], whi = a.col_whi[c];
  double tot = a.pieces[2 * wlo + 1];
  for (int w = wlo + 1; w < whi; ++w) tot += a.pieces[2 * w];
  tot += a.pieces[2 * whi];
  return tot;
}

struct TrialCtl {
  bool init, lead;
  int xi;
};

template <int NT, int THREADS = kThreads, int ST = ST_F32>
__device__ __forceinline__ void trial_store(const FwdArgs& a, int i0, const TrialRegs<NT>& R, const TrialCtl& T,
                                            const double (&lam)[NT], float* xs, double (&sq)[NT]) {
  const int nb = a.nb, nbp = pad4(nb);
#pragma unroll
  for (int u = 0; u < kTrialU; ++u) {
    const int i = i0 + u * THREADS;
    if (i >= nb) continue;
    float x = R.xc[0][u];
#pragma unroll
    // x_k is the candidate the state names.  Blended with exact 0/1 weights
    // rather than selected: a select among elements of the candidate array
    // becomes an indexed load from a stack copy of it (scratch memory).  The
    // candidates are finite: each solve starts with the other iterate
    // buffers zeroed, and a non-finite trial ends the solve.
    for (int j = 1; j <= NT; ++j) {
      const float c = (T.xi == j) ? 1.0f : 0.0f;
      x = x * (1.0f - c) + R.xc[j][u] * c;
    }
    if (T.init) {
#pragma unroll
      for (int q = 0; q < NT; ++q) xs[q * nbp + i] = !coded(ST) ? x : x * R.sc[u];
      continue;
    }
    const double gf = !coded(ST) ? a.g_scale : a.g_scale * static_cast<double>(R.sc[u]);
    float g = R.g[u];
    if (R.kind[u] == 1) g = static_cast<float>(gf * (R.p0[u] + R.p1[u]));
    else if (R.kind[u] > 1) g = static_cast<float>(gf * pieces_sum(a, i));
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const float t = trial_point(x, g, lam[q]);
      xs[q * nbp + i] = !coded(ST) ? t : t * R.sc[u];
      if (T.lead) {
        select_buf(a.xbuf, (T.xi + 1 + q) % (NT + 1))[i] = t;
        const double dl = static_cast<double>(t) - static_cast<double>(x);
        sq[q] += dl * dl;
      }
    }
  }
}

// After the first round (loaded by the caller): the remaining rounds, the
// lead workgroup's step norms, the penalty table; ends with a barrier.
template <int NT, int THREADS = kThreads, int ST = ST_F32>
__device__ __forceinline__ void trial_finish(const FwdArgs& a, const TrialRegs<NT>& R, const TrialCtl& T,
                                             const double (&lam)[NT], PenaltyDev* tab, float* xs, double* red,
                                             int G) {
  const int tid = threadIdx.x;
  double sq[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) sq[q] = 0.0;
  {
    double* dst = reinterpret_cast<double*>(tab);
    if (tid < 4 * a.nstruct) dst[tid] = R.tab;
    for (int i = tid + THREADS; i < 4 * a.nstruct; i += THREADS)
      dst[i] = reinterpret_cast<const double*>(a.pen.table)[i];
  }
  trial_store<NT, THREADS, ST>(a, tid, R, T, lam, xs, sq);
  for (int i0 = tid + kTrialU * THREADS; i0 < a.nb; i0 += kTrialU * THREADS) {
    TrialRegs<NT> R2;
    trial_load<NT, THREADS, ST>(a, i0, R2);
    trial_store<NT, THREADS, ST>(a, i0, R2, T, lam, xs, sq);
  }
  if (T.lead && !T.init) {
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const double t = block_sum<double, THREADS / 64>(sq[q], red);
      if (tid == 0) a.partials[NT * G + q] = t;
    }
  }
  __syncthreads();
}

template <int NT, int THREADS = kThreads>
__device__ __forceinline__ void stage_inputs(const FwdArgs& a, const float* src, PenaltyDev* tab, float* xs,
                                             bool want_sid) {
  StageRegs<NT> R;
  stage_start<NT, THREADS>(a, src, want_sid, R);
  stage_finish<NT, THREADS>(a, src, want_sid, R, tab, xs);
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
  float* prod = xs + NT * nbp;
  int32_t* rp = reinterpret_cast<int32_t*>(prod + NT * kFwdNnzMax);
  uint8_t* sidl = reinterpret_cast<uint8_t*>(rp + kFwdRowsMax + 1);
  __shared__ double red[kWaves];
  __shared__ float redf[kWaves];

  const int tid = threadIdx.x;
  const bool solve = (a.mode == FWD_SOLVE);
  const bool want_sid = (a.mode != FWD_PLAIN);
  int ntr = 1;
  float* rout[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) rout[q] = nullptr;
  TrialCtl T{true, false, 0};
  double lam[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) lam[q] = 0.0;
  if (solve) {
    const SolverState* st = a.st_in;
    // the state passes through unchanged (word copy by workgroup 0)
    constexpr int kWords = static_cast<int>(sizeof(SolverState) / sizeof(int32_t));
    if (blockIdx.x == 0 && tid < kWords)
      reinterpret_cast<int32_t*>(a.st_out)[tid] = reinterpret_cast<const int32_t*>(st)[tid];
    const int phase = st->phase;
    if (phase == PH_DONE) return;
    ntr = (phase == PH_INIT) ? 1 : NT;
    T.init = (phase == PH_INIT);
    T.lead = (blockIdx.x == 0);
    T.xi = st->xi;
    lam[0] = st->lambda;
    const double alpha = st->alpha;
#pragma unroll
    for (int q = 1; q < NT; ++q) lam[q] = lam[q - 1] / alpha;
#pragma unroll
    for (int q = 0; q < NT; ++q) rout[q] = a.rbuf[q];
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

  if (solve) {
    TrialRegs<NT> TR;
    trial_load<NT>(a, tid, TR);
    TR.tab = (tid < 4 * a.nstruct) ? reinterpret_cast<const double*>(a.pen.table)[tid] : 0.0;
    trial_finish<NT>(a, TR, T, lam, tab, xs, red, gridDim.x);
  } else {
    stage_inputs<NT>(a, a.x, tab, xs, want_sid);
  }

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
// Each of the four waves of a workgroup streams its own contiguous range of
// small row blocks (at most wave_part_nnz nonzeros and kWaveRowsMax rows),
// an even split of the block count (a block's time is mostly latency, so
// equal counts balance better than equal bytes).
// Block bounds come from per-lane copies of the block table read with
// readlane, so all control flow and every descriptor is wave-uniform.  A
// block's column indices and values arrive as 16-byte buffer loads (lanes
// past the block read zeros), its products D_ij x_j go to the wave's LDS
// region, and groups of L lanes (the largest power of two with L * rows <= 64)
// sum one row each, reading four products per round and combining the lanes
// with DPP moves.  Row pointers and structure ids of a row are loaded by the
// lane that finishes it.  The next block's loads are issued as soon as the
// products of the current one are in LDS.
constexpr int kWaveSlack = 256;   // LDS floats after the last wave region (over-reads of masked slots)

// Groups of four entries per lane in one wave's row block: 2 (512 entries)
// with float32 storage, 3 (768) with float32 values and 16-bit indices, 4
// (1024 entries) with 16-bit storage.
template <int ST>
constexpr int wave_groups() { return wave_nnz(ST) / 256; }

template <int ST>
struct WaveStage {
  ColGroup<ST> c[wave_groups<ST>()];
  ValGroup<ST> v[wave_groups<ST>()];
  int rlo[kWavePasses], rhi[kWavePasses];
  uint32_t sid[kWavePasses];
};

// Loads of the entries base + 4 lane + 256 j + u (u < 4, j < the group count)
// of the CSR index and value arrays; base is a multiple of 4 and the arrays
// carry a zeroed tail, so whole groups stay in bounds and entries past k1
// read zeros.
template <int ST, int CP = 0>
__device__ __forceinline__ void csr_issue(const FwdArgs& a, int base, int k1, int lane,
                                          ColGroup<ST> (&c)[wave_groups<ST>()],
                                          ValGroup<ST> (&v)[wave_groups<ST>()]) {
  constexpr int G = wave_groups<ST>();
  if constexpr (ST == ST_F32) {
    const uint32_t bytes = static_cast<uint32_t>((k1 - base) * 4 + 15) & ~15u;
    const rsrc_t rc = make_rsrc(a.col_idx + base, bytes);
    const rsrc_t rv = make_rsrc(a.val + base, bytes);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      c[j] = load_i4s<CP>(rc, 16 * lane + 1024 * j);
      v[j] = load_f4s<CP>(rv, 16 * lane + 1024 * j);
    }
  } else if constexpr (ST == ST_F32C16) {
    const uint32_t n = static_cast<uint32_t>(k1 - base);
    const rsrc_t rc = make_rsrc(a.col16 + base, (n * 2 + 7) & ~7u);
    const rsrc_t rv = make_rsrc(a.val + base, (n * 4 + 15) & ~15u);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      c[j] = load_u2s<CP>(rc, 8 * lane + 512 * j);
      v[j] = load_f4s<CP>(rv, 16 * lane + 1024 * j);
    }
  } else {
    const uint32_t bytes = static_cast<uint32_t>((k1 - base) * 2 + 7) & ~7u;
    const rsrc_t rc = make_rsrc(a.col16 + base, bytes);
    const rsrc_t rv = make_rsrc(a.val16 + base, bytes);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      c[j] = load_u2s<CP>(rc, 8 * lane + 512 * j);
      v[j] = load_u2s<CP>(rv, 8 * lane + 512 * j);
    }
  }
}

struct WaveBlock {
  int r0, r1, k0, k1;
};

__device__ __forceinline__ int log2_lanes(int nr) {
  // largest L = 2^e <= 64 with L * nr <= 64 (L = 1 beyond 64 rows)
  int e = 6;
  while (e > 0 && (nr << e) > 64) --e;
  return e;
}

// UNCOND: every row load is issued (rows past the block read zeros out of
// bounds), so that no load of the block sits in a branch and a later wait
// for an earlier load can count exactly how many were issued after it.
template <int MODE, bool UNCOND = false, int ST = ST_F32, int CP = 0>
__device__ __forceinline__ void wave_issue(const FwdArgs& a, const WaveBlock& m, int lane, WaveStage<ST>& S) {
  csr_issue<ST, CP>(a, m.k0 & ~3, m.k1, lane, S.c, S.v);
  const int nr = m.r1 - m.r0;
  const int e = log2_lanes(nr);
  const int passes = ((nr << e) + 63) >> 6;
  const rsrc_t rp = make_rsrc(a.row_ptr + m.r0, static_cast<uint32_t>(nr + 1) * 4);
  const rsrc_t rs = make_rsrc(a.pen.sid + m.r0, static_cast<uint32_t>(nr));
#pragma unroll
  for (int p = 0; p < kWavePasses; ++p) {
    S.rlo[p] = S.rhi[p] = 0;
    S.sid[p] = 0;
    if (UNCOND) {
      const int row = (p < passes) ? (p << (6 - e)) + (lane >> e) : nr + 1;
      S.rlo[p] = load_i32(rp, 4 * row);
      S.rhi[p] = load_i32(rp, 4 * row + 4);
      if (MODE != FWD_PLAIN) S.sid[p] = load_u8(rs, row);
    } else if (p < passes) {
      const int row = (p << (6 - e)) + (lane >> e);
      S.rlo[p] = load_i32(rp, 4 * row);
      S.rhi[p] = load_i32(rp, 4 * row + 4);
      if (MODE != FWD_PLAIN) S.sid[p] = load_u8(rs, row);
    }
  }
}

template <int NT, int MODE>
__device__ __forceinline__ void row_finish(const FwdArgs& a, int row, uint32_t sid, const PenaltyDev* tab,
                                           const float (&d)[NT], double (&pacc)[NT], const rsrc_t (&rout)[NT],
                                           const rsrc_t& dout, int ntr) {
#pragma clang fp contract(off)
  const uint32_t off = 4u * static_cast<uint32_t>(row);
  if (MODE == FWD_PLAIN) {
    store_f32(dout, off, d[0]);
    pacc[0] += static_cast<double>(d[0]) * static_cast<double>(d[0]);
    return;
  }
  const RowPenalty pen = row_penalty(a.pen, row, tab, static_cast<uint8_t>(sid));
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    if (q < ntr) {
      double F;
      float r;
      penalty(pen, d[q], F, r);
      pacc[q] += F;
      if (MODE == FWD_SOLVE) {
        store_f32(rout[q], off, r);
      } else if (q == 0) {
        if (a.r_out) store_f32(rout[0], off, r);
        if (a.d_out) store_f32(dout, off, d[0]);
      }
    }
  }
}

// Row sums of one block with L lanes per row.
template <int L, int NT, int MODE, int NNZ, typename WS>
__device__ __forceinline__ void wave_rows(const FwdArgs& a, const float* prod, int lane, const WaveBlock& m,
                                          const WS& S, const PenaltyDev* tab, double (&pacc)[NT],
                                          const rsrc_t (&rout)[NT], const rsrc_t& dout, int ntr) {
  constexpr int kRowsPerPass = 64 / L;
  const int a0 = m.k0 & ~3;
  const int nr = m.r1 - m.r0;
  const int passes = (nr * L + 63) / 64;
  const int sub = lane & (L - 1);
#pragma unroll
  for (int p = 0; p < kWavePasses; ++p) {
    if (p < passes) {
      const int row = p * kRowsPerPass + lane / L;
      const int s1 = S.rhi[p] - a0;
      float acc[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) acc[q] = 0.f;
      // rounds of four products per lane: whole rounds first, then at most
      // one round that runs past the row's end (its tail slots read as zero)
      int k = S.rlo[p] - a0 + sub;
      for (; k + 3 * L < s1; k += 4 * L) {
#pragma unroll
        for (int q = 0; q < NT; ++q) {
          const float* pq = prod + q * NNZ + k;
          acc[q] += (pq[0] + pq[L]) + (pq[2 * L] + pq[3 * L]);
        }
      }
      if (k < s1) {
        const int left = s1 - k;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
          const float* pq = prod + q * NNZ + k;
          float v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float t = pq[u * L];   // always in the allocation; masked below
            v[u] = (u * L < left) ? t : 0.0f;
          }
          acc[q] += (v[0] + v[1]) + (v[2] + v[3]);
        }
      }
      float d[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) d[q] = group_sum<L>(acc[q]);
      if (sub == L - 1 && row < nr) row_finish<NT, MODE>(a, m.r0 + row, S.sid[p], tab, d, pacc, rout, dout, ntr);
    }
  }
}

// Waves of a wave-granular forward workgroup: sixteen, one workgroup per
// compute unit, for a matrix solved alone; eight, up to three side by side,
// once per-plan targets are applied for dispatches that several plans share
// (one workgroup's staging -- the start of every workgroup, and of every
// plan's workgroups in a batched pass -- then overlaps the others'
// streams).  Launch bounds: 8-wave workgroups with one and two trials per
// pass keep within 80 and 128 registers per lane (six and four waves per
// SIMD); four trials take 8-wave workgroups with no such bound.
template <int NT, int WAVES>
constexpr int fwd_min_waves_per_simd() { return WAVES == 16 ? 4 : NT == 1 ? 6 : NT == 2 ? 4 : 1; }
constexpr int kMetaChunk = 256;   // row blocks whose bounds are staged in LDS at a time

template <int NT, int MODE, int WAVES, int ST, int CP = 0>
__device__ __forceinline__ void fwd_wave_pass(const FwdArgs& a, const Slot sl) {
  constexpr int THREADS = WAVES * 64;
  constexpr int NNZ = wave_nnz(ST), PART = wave_part_nnz(ST), NG = wave_groups<ST>();
  extern __shared__ __align__(16) unsigned char smem[];
  const int nb = a.nb;
  const int nbp = pad4(nb);
  PenaltyDev* tab = reinterpret_cast<PenaltyDev*>(smem);
  float* xs = reinterpret_cast<float*>(tab + a.nstruct);
  float* prod0 = xs + NT * nbp;
  int32_t* mrow = reinterpret_cast<int32_t*>(prod0 + WAVES * NT * NNZ + kWaveSlack);
  int32_t* mk0 = mrow + (kMetaChunk + 1);
  int32_t* mend = mk0 + (kMetaChunk + 1);
  double* gpart = reinterpret_cast<double*>(mend + kMetaChunk + 2);   // 8-byte aligned
  const int wv = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  float* prod = prod0 + wv * (NT * NNZ);
  __shared__ double red[WAVES];
  __shared__ int next_blk;

  const int tid = threadIdx.x;
  constexpr bool solve = (MODE == FWD_SOLVE);
  constexpr bool want_sid = (MODE != FWD_PLAIN);

  // This workgroup's contiguous range of row blocks; its waves take blocks
  // in turn from a counter in LDS (the first WAVES blocks one each), so a
  // wave that runs faster takes more.  Every block's objective contribution
  // goes to its own LDS slot and the workgroup adds the slots in block order,
  // so the total does not depend on which wave took which block.
  const int G = sl.G, w = sl.w;
  const int lw = (G % kXcds == 0) ? (w % kXcds) * (G / kXcds) + w / kXcds : w;
  const int B0 = split_point(lw, a.nwblocks, G);
  const int B1 = split_point(lw + 1, a.nwblocks, G);
  // Loads in the order their results are needed, none of them in a branch:
  // the first block's bounds (lanes 0 and 1), the staging inputs (a solve's
  // trial inputs before the state is known), the state (one word per lane),
  // then the first block's nonzeros.  So no wait for one of them waits for a
  // later one, and the block's loads overlap the staging.
  int b = B0 + wv;
  const bool first = b < min(B1, B0 + kMetaChunk);
  const uint32_t meta_bytes = 4u * static_cast<uint32_t>(a.nwblocks + 1);
  const uint32_t moff = 4u * static_cast<uint32_t>(b + (lane & 1));
  const int mrow0 = load_i32(make_rsrc(a.wblock_row, meta_bytes), 4u * static_cast<uint32_t>(b));
  const int mend0 = load_i32(make_rsrc(a.wblock_end, meta_bytes - 4u), 4u * static_cast<uint32_t>(b));
  const int mk00 = load_i32(make_rsrc(a.wblock_k0, meta_bytes), moff);
  // the first chunk's block bounds (thread i loads entry B0 + i), stored to
  // LDS before the staging barrier, so that no round trip and no barrier of
  // their own stand between the staging and the first block
  static_assert(THREADS > kMetaChunk, "one thread per bound of the first chunk");
  const int cfirst = min(B1, B0 + kMetaChunk) - B0;
  const uint32_t mi = 4u * static_cast<uint32_t>(B0 + tid);
  const int pre_row = load_i32(make_rsrc(a.wblock_row, meta_bytes), mi);
  const int pre_k0 = load_i32(make_rsrc(a.wblock_k0, meta_bytes), mi);
  const int pre_end = load_i32(make_rsrc(a.wblock_end, meta_bytes - 4u), mi);
  TrialRegs<NT> TR;
  StageRegs<NT> SR;
  int32_t sw = 0;
  if (solve) {
    trial_load<NT, THREADS, ST>(a, tid, TR);
    TR.tab = load_f64(make_rsrc(a.pen.table, 32u * static_cast<uint32_t>(a.nstruct)), 8u * tid);
    sw = reinterpret_cast<const int32_t*>(a.st_in)[lane < kStateWords ? lane : 0];
  } else {
    stage_start<NT, THREADS, ST>(a, a.x, want_sid, SR);
  }
  WaveBlock cur{0, 0, 0, 0};
  if (first) {
    cur.r0 = __builtin_amdgcn_readlane(mrow0, 0);
    cur.r1 = __builtin_amdgcn_readlane(mend0, 0);
    cur.k0 = __builtin_amdgcn_readlane(mk00, 0);
    cur.k1 = __builtin_amdgcn_readlane(mk00, 1);
  }
  // a row longer than a wave block is streamed in the loop instead
  const bool short_first = cur.k1 - cur.k0 <= PART;
  WaveStage<ST> S;
  wave_issue<MODE, true, ST, CP>(a, short_first ? cur : WaveBlock{0, 0, 0, 0}, lane, S);

  int ntr = 1;
  rsrc_t rout[NT];
  const uint32_t vbytes = 4u * static_cast<uint32_t>(a.nv);
#pragma unroll
  for (int q = 0; q < NT; ++q) rout[q] = make_rsrc(a.r_out, a.r_out ? vbytes : 0u);
  const rsrc_t dout = make_rsrc(a.d_out, a.d_out ? vbytes : 0u);
  TrialCtl T{true, false, 0};
  double lam[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) lam[q] = 0.0;
  if (solve) {
    if (sl.w == 0 && wv == 0 && lane < kStateWords) reinterpret_cast<int32_t*>(a.st_out)[lane] = sw;
    const int phase = state_int(sw, offsetof(SolverState, phase));
    if (phase == PH_DONE) return;
    ntr = (phase == PH_INIT) ? 1 : NT;
    T.init = (phase == PH_INIT);
    T.lead = (sl.w == 0);
    T.xi = state_int(sw, offsetof(SolverState, xi));
    lam[0] = state_f64(sw, offsetof(SolverState, lambda));
    const double alpha = state_f64(sw, offsetof(SolverState, alpha));
#pragma unroll
    for (int q = 1; q < NT; ++q) lam[q] = lam[q - 1] / alpha;
#pragma unroll
    for (int q = 0; q < NT; ++q) rout[q] = make_rsrc(a.rbuf[q], vbytes);
  }
  if (tid <= cfirst) {
    mrow[tid] = pre_row;
    mk0[tid] = pre_k0;
    if (tid < cfirst) mend[tid] = pre_end;
  }
  if (tid == 0) next_blk = B0 + WAVES;
  // (both stagings end with a barrier)
  if (solve) trial_finish<NT, THREADS, ST>(a, TR, T, lam, tab, xs, red, sl.G);
  else stage_finish<NT, THREADS, ST>(a, a.x, want_sid, SR, tab, xs);

  double gsum[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) gsum[q] = 0.0;
  for (int c0 = B0; c0 < B1; c0 += kMetaChunk) {
    const int c1 = min(c0 + kMetaChunk, B1);
    if (c0 != B0) {
      for (int i = tid; i <= c1 - c0; i += THREADS) {
        mrow[i] = a.wblock_row[c0 + i];
        mk0[i] = a.wblock_k0[c0 + i];
        if (i < c1 - c0) mend[i] = a.wblock_end[c0 + i];
      }
      if (tid == 0) next_blk = c0 + WAVES;
      __syncthreads();
    }
    auto meta = [&](int blk) {
      const int i = blk - c0;
      WaveBlock m;
      m.r0 = uniform(mrow[i]);
      m.r1 = uniform(mend[i]);
      m.k0 = uniform(mk0[i]);
      m.k1 = uniform(mk0[i + 1]);
      return m;
    };
    if (c0 != B0) {
      b = c0 + wv;
      cur = (b < c1) ? meta(b) : WaveBlock{0, 0, 0, 0};
      wave_issue<MODE, true, ST, CP>(a, (b < c1 && cur.k1 - cur.k0 <= PART) ? cur : WaveBlock{0, 0, 0, 0}, lane, S);
    }
    while (b < c1) {
      // the block after this one (taken now, its loads issued once this
      // block's products are in LDS)
      int nxt = 0;
      if (lane == 0) nxt = atomicAdd(&next_blk, 1);
      nxt = uniform(nxt);
      const WaveBlock blk = cur;
      const bool more = nxt < c1;
      if (more) cur = meta(nxt);
      double pb[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) pb[q] = 0.0;
      if (blk.k1 - blk.k0 > PART) {
        // one row longer than a wave block: the wave strides over it
        float acc[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[q] = 0.f;
        for (int base = blk.k0 & ~3; base < blk.k1; base += NNZ) {
          ColGroup<ST> cg[NG];
          ValGroup<ST> vg[NG];
          csr_issue<ST, CP>(a, base, blk.k1, lane, cg, vg);
#pragma unroll
          for (int j = 0; j < NG; ++j) {
            const int e0 = base + 4 * lane + 256 * j;
#pragma unroll
            for (int q = 0; q < NT; ++q) {
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const float t = val_of<ST>(vg[j], u) * xs[q * nbp + col_of(cg[j], u)];
                acc[q] += (e0 + u >= blk.k0 && e0 + u < blk.k1) ? t : 0.0f;
              }
            }
          }
        }
        float d[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) d[q] = wave_sum(acc[q]);
        if (lane == 63) {
          const uint32_t sid = want_sid ? a.pen.sid[blk.r0] : 0;
          row_finish<NT, MODE>(a, blk.r0, sid, tab, d, pb, rout, dout, ntr);
        }
        wave_issue<MODE, true, ST, CP>(a, (more && cur.k1 - cur.k0 <= PART) ? cur : WaveBlock{0, 0, 0, 0}, lane, S);
      } else {
        // products of this block into the wave's LDS region (lanes past the
        // block hold zeros and write slots that no row reads)
#pragma unroll
        for (int j = 0; j < NG; ++j) {
          const int off = 4 * lane + 256 * j;
#pragma unroll
          for (int q = 0; q < NT; ++q) {
            const float* xq = xs + q * nbp;
            float4 p;
            p.x = val_of<ST>(S.v[j], 0) * xq[col_of(S.c[j], 0)];
            p.y = val_of<ST>(S.v[j], 1) * xq[col_of(S.c[j], 1)];
            p.z = val_of<ST>(S.v[j], 2) * xq[col_of(S.c[j], 2)];
            p.w = val_of<ST>(S.v[j], 3) * xq[col_of(S.c[j], 3)];
            *reinterpret_cast<float4*>(prod + q * NNZ + off) = p;
          }
        }
        // LDS operations of one wave complete in order; the fence only keeps
        // the compiler from moving the row reads above the product writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const WaveStage<ST> R = S;   // this block's row pointers and ids (loads already waited on)
        // issued whether or not a next block follows (an empty block reads
        // zeros and touches no memory), so the loads land in the registers
        // the next products read, with no copies to merge two paths
        wave_issue<MODE, true, ST, CP>(a, (more && cur.k1 - cur.k0 <= PART) ? cur : WaveBlock{0, 0, 0, 0}, lane, S);
        switch (log2_lanes(blk.r1 - blk.r0)) {
          case 0: wave_rows<1, NT, MODE, NNZ>(a, prod, lane, blk, R, tab, pb, rout, dout, ntr); break;
          case 1: wave_rows<2, NT, MODE, NNZ>(a, prod, lane, blk, R, tab, pb, rout, dout, ntr); break;
          case 2: wave_rows<4, NT, MODE, NNZ>(a, prod, lane, blk, R, tab, pb, rout, dout, ntr); break;
          case 3: wave_rows<8, NT, MODE, NNZ>(a, prod, lane, blk, R, tab, pb, rout, dout, ntr); break;
          case 4: wave_rows<16, NT, MODE, NNZ>(a, prod, lane, blk, R, tab, pb, rout, dout, ntr); break;
          case 5: wave_rows<32, NT, MODE, NNZ>(a, prod, lane, blk, R, tab, pb, rout, dout, ntr); break;
          default: wave_rows<64, NT, MODE, NNZ>(a, prod, lane, blk, R, tab, pb, rout, dout, ntr); break;
        }
        // the next block's LDS writes must not overtake this block's reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const double t = wave_sum(pb[q]);
        if (lane == 63) gpart[q * kMetaChunk + (b - c0)] = t;
      }
      b = nxt;
    }
    __syncthreads();
    if (wv == 0) {
      // the chunk's block contributions in a fixed order: lane l adds blocks
      // l, l + 64, ..., then the lanes are summed
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        double t = 0.0;
        for (int i = lane; i < c1 - c0; i += 64) t += gpart[q * kMetaChunk + i];
        gsum[q] += wave_sum(t);
      }
    }
    __syncthreads();
  }
  if (wv == 0 && lane == 63) {
#pragma unroll
    for (int q = 0; q < NT; ++q) a.partials[q * sl.G + sl.w] = gsum[q];
  }
}

template <int NT, int MODE, int WAVES, int ST, int CP = 0>
__global__ __launch_bounds__(WAVES * 64, (fwd_min_waves_per_simd<NT, WAVES>())) void fwd_wave_kernel(FwdArgs a) {
  fwd_wave_pass<NT, MODE, WAVES, ST, CP>(a, Slot{static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x)});
}

// Batched solve pass: slots[blockIdx.x] = (plan << 16) | workgroup of that
// plan's pass, or -1 for an idle slot (plans start at multiples of the die
// count, so each plan keeps its workgroups' die placement).
template <int NT, int WAVES, int ST, int CP = 0>
__global__ __launch_bounds__(WAVES * 64, (fwd_min_waves_per_simd<NT, WAVES>())) void fwd_wave_batch_kernel(const FwdArgs* __restrict__ args,
                                                                    const int32_t* __restrict__ slots) {
  const int sv = uniform(slots[blockIdx.x]);
  if (sv < 0) return;
  const FwdArgs& a = args[sv >> 16];
  fwd_wave_pass<NT, FWD_SOLVE, WAVES, ST, CP>(a, Slot{sv & 0xFFFF, a.grid});
}

// ---- adjoint pass ----------------------------------------------------------------
// Workgroup w owns nonzeros [k0w, k1w) of the CSC arrays and walks the tiles
// covering them in rounds of 2048 entries: each thread loads two 16-byte
// vectors of row indices and of values, i.e. entries e0 + 1024 j + 64 u
// (j < 2, u < 4) of the round, where e0 = 256 * wave + lane (the tiled slot
// order of the CSC arrays); lanes past the range read zeros.  A round's
// residual gathers (each a run of 64 consecutive entries of a column across
// the wave) are issued before the next round's loads, which go to the other
// of two register stages, so one round is always in flight.  A round inside
// one column adds all its products; a round that meets a column boundary adds
// each column's share under a mask and closes every column that ends in it.
template <int ST>
struct AdjStage {
  int4 c[2];
  ValGroup<ST> v[2];
};

constexpr int kAdjStep = 8 * kThreads;   // nonzeros per round

// Logical workgroup of this dispatch slot.  With xcd_map and a grid that is a
// multiple of the die count, workgroup w (on die w % 8) gets logical slot
// (w % 8) * (grid / 8) + w / 8, so each die owns one contiguous eighth.
__device__ __forceinline__ int logical_wg(const Slot sl, bool xcd_map) {
  const int G = sl.G, w = sl.w;
  return (xcd_map && G % kXcds == 0) ? (w % kXcds) * (G / kXcds) + w / kXcds : w;
}

// rv covers the value array from the same entry as ri: float32 values in
// the index slots' order, or 16-bit codes in that order at half the width.
template <int ST, int CP = 0>
__device__ __forceinline__ void adj_issue(rsrc_t ri, rsrc_t rv, int round, AdjStage<ST>& S) {
  const uint32_t t = 16u * threadIdx.x;
  const uint32_t base = static_cast<uint32_t>(round) * (kAdjStep * 4u);
#pragma unroll
  for (int j = 0; j < 2; ++j) S.c[j] = load_i4s<CP>(ri, base + t + 4096u * j);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if constexpr (ST == ST_F32) S.v[j] = load_f4s<CP>(rv, base + t + 4096u * j);
    else S.v[j] = load_u2s<CP>(rv, base / 2 + t / 2 + 2048u * j);
  }
}

template <typename AS>
__device__ __forceinline__ void adj_gather(rsrc_t rr, const AS& S, float (&g)[8]) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    g[4 * j + 0] = load_f32(rr, 4u * S.c[j].x);
    g[4 * j + 1] = load_f32(rr, 4u * S.c[j].y);
    g[4 * j + 2] = load_f32(rr, 4u * S.c[j].z);
    g[4 * j + 3] = load_f32(rr, 4u * S.c[j].w);
  }
}

// Float64 sum of this thread's eight products, in a fixed order.
template <int ST>
__device__ __forceinline__ double adj_dot(const AdjStage<ST>& S, const float (&g)[8]) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int u = 0; u < 4; ++u) s += static_cast<double>(val_of<ST>(S.v[j], u)) * static_cast<double>(g[4 * j + u]);
  }
  return s;
}

// The same over the entries with index in [lo, hi) (e0 as above).
template <int ST>
__device__ __forceinline__ double adj_dot_masked(const AdjStage<ST>& S, const float (&g)[8], int e0, int lo, int hi) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + 1024 * j + 64 * u;
      const float r = (e >= lo && e < hi) ? g[4 * j + u] : 0.0f;
      s += static_cast<double>(val_of<ST>(S.v[j], u)) * static_cast<double>(r);
    }
  }
  return s;
}

// ---- an adjoint workgroup's columns ----------------------------------------------
// A workgroup walks its columns c0..c1-1 in order, kColChunk at a time: lane
// j of every wave holds column cb + j's entries of col_ptr (and its kind and
// 16-bit scale), so moving on to the next column reads a register.  Closing a
// column sums it over each wave and parks the wave's sum in lane j; when the
// chunk is full, and at the end, the waves' sums meet in LDS and wave 0 adds
// them in wave order (block_sum's order) and stores the chunk's gradient
// entries and pieces.  No workgroup barrier and no dependent global load sits
// between one column and the next.
constexpr int kColChunk = 64;

template <int ST>
struct ColChunk {
  int cb;          // first column of the chunk (uniform)
  int p0, p1;      // lane j: col_ptr[cb + j], col_ptr[cb + j + 1]
  uint32_t kind;   // lane j: col_kind[cb + j]
  float csc;       // lane j: 16-bit storage scale of column cb + j
};

template <int ST>
__device__ __forceinline__ void col_chunk_load(const AdjArgs& a, int cb, ColChunk<ST>& K) {
  const uint32_t nb = static_cast<uint32_t>(a.nb);
  const uint32_t j = static_cast<uint32_t>(cb + (threadIdx.x & 63));
  const rsrc_t rp = make_rsrc(a.col_ptr, 4u * (nb + 1));
  K.cb = cb;
  K.p0 = load_i32(rp, 4u * j);
  K.p1 = load_i32(rp, 4u * j + 4u);
  K.kind = load_u8(make_rsrc(a.col_kind, nb), j);
  K.csc = coded(ST) ? load_f32(make_rsrc(a.col_scale, 4u * nb), 4u * j) : 1.0f;
}

// Loads of a chunk after the first one: wait for them at once (vmcnt 0).
// Without this wait, the compiler cannot tell at the next column whether a
// reload is still in flight, and every column's register read would wait
// for all loads issued since, the next round's prefetch included.
constexpr int kWaitVmcnt0 = 0x0F70;   // vmcnt 0, expcnt and lgkmcnt unchecked

template <int ST>
__device__ __forceinline__ void col_chunk_reload(const AdjArgs& a, int cb, ColChunk<ST>& K) {
  col_chunk_load(a, cb, K);
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
}

// Column c's entries inside the workgroup's range [k0w, k1w).
template <int ST>
__device__ __forceinline__ void col_bounds(const ColChunk<ST>& K, int c, int k0w, int k1w, int& lo, int& hi) {
  lo = max(__builtin_amdgcn_readlane(K.p0, c - K.cb), k0w);
  hi = min(__builtin_amdgcn_readlane(K.p1, c - K.cb), k1w);
}

// The wave's sum of v, parked in lane j of h.
__device__ __forceinline__ void col_park(double v, int j, double& h) {
  const uint64_t b = __builtin_bit_cast(uint64_t, wave_sum(v));
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b), 63));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), 63));
  if ((threadIdx.x & 63) == j) h = __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// Lane j of wave 0, column c = cb + j closed with workgroup sum t: the
// gradient entry of a column inside the range, else the workgroup's piece.
template <int ST>
__device__ __forceinline__ void col_store(const AdjArgs& aq, const ColChunk<ST>& K, int c0, int c1, int lw, int k0w,
                                          int k1w, double t) {
  const int c = K.cb + (threadIdx.x & 63);
  if (K.p0 >= k0w && K.p1 <= k1w) {
    const double f = (ST == ST_F32) ? aq.scale : aq.scale * static_cast<double>(K.csc);
    aq.out[c] = static_cast<float>(f * t);
  } else {
    if (c == c0) aq.pieces[2 * lw] = t;
    if (c == c1 - 1) aq.pieces[2 * lw + 1] = t;
    // a column shared by two workgroups also keeps its pieces side by side
    if (K.kind == 1 && aq.pieces_col != nullptr) aq.pieces_col[2 * c + (K.p0 < k0w ? 1 : 0)] = t;
  }
}

// Adjoint pass: in a solve, the decision on the preceding forward pass
// (every workgroup identically; workgroup 0 stores the new state and trace
// entry), and g = scale * D^T r over this workgroup's share of the nonzeros.
// The first two rounds' loads are issued on entry and the first round's
// residual gathers before the decision is known, from the residual buffer of
// the pass's first trial (the one an accepted step of a single-trial pass
// always lands in); if another trial is accepted they are issued again.
template <int NT, bool SOLVE, int ST, int CP = 0>
__device__ __forceinline__ void adj_pass(const AdjArgs& a, const Slot sl) {
  __shared__ double red[kWaves];
  __shared__ double colsh[kWaves * kColChunk];
  __shared__ Decision dec;
  const int tid = threadIdx.x;
  const int lw = logical_wg(sl, a.xcd_map != 0);
  const int k0w = split_point(lw, static_cast<int>(a.nnz), a.grid);
  const int k1w = split_point(lw + 1, static_cast<int>(a.nnz), a.grid);
  const int kb = k0w & ~(kTile - 1);
  const int nrounds = (k1w > kb) ? (k1w - kb + kAdjStep - 1) / kAdjStep : 0;
  // whole tiles: entries of a partial tile sit anywhere in it
  const uint32_t bytes = static_cast<uint32_t>((((k1w + kTile - 1) & ~(kTile - 1)) - kb) * 4);
  const rsrc_t ri = make_rsrc(a.row_idx + kb, bytes);
  const rsrc_t rv = (ST == ST_F32) ? make_rsrc(a.val + kb, bytes) : make_rsrc(a.val16 + kb, bytes / 2);
  // Every load of the prologue is issued at once and none sits in a branch
  // (rounds past the range read zeros out of bounds), so each wait below
  // waits for its own loads only: the decision's inputs, this workgroup's
  // columns, the first two rounds, then the gathers of the first round.
  DecideLoads<NT> DL;
  if (SOLVE) decide_start<NT>(a, DL);
  const int4 wi = load_i4(make_rsrc(a.wg_cols, 16u * static_cast<uint32_t>(a.grid)), 16u * static_cast<uint32_t>(lw));
  AdjStage<ST> A, B;
  adj_issue<ST, CP>(ri, rv, 0, A);
  adj_issue<ST, CP>(ri, rv, 1, B);
  const int c0 = uniform(wi.x), c1 = uniform(wi.y);
  int c = c0, lo = uniform(wi.z), hi = uniform(wi.w);
  ColChunk<ST> CK;
  col_chunk_load(a, c0, CK);
  // a solve gathers the residual of the first trial: the accepted one
  // unless a later trial wins
  const uint32_t rbytes = 4u * static_cast<uint32_t>(a.nv);
  rsrc_t rr = make_rsrc(SOLVE ? a.rbuf[0] : a.r, rbytes);
  float g[8];
  adj_gather(rr, A, g);
  if (SOLVE) {
    // (a finished solve passes its state through unchanged and exits here)
    decide<NT>(a.fwd_partials, a.fwd_parts, a.step_partials, a.step_parts, DL, dec, red, a.G_skip);
    if (sl.w == 0 && tid == 0) {
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
    if (dec.st.acc != 0) {
      rr = make_rsrc(select_buf(a.rbuf, dec.st.acc), rbytes);
      adj_gather(rr, A, g);
    }
  }

  double s = 0.0, h = 0.0;
  // the chunk's closed columns: the waves' sums in wave order, then stored
  auto flush = [&]() {
    colsh[(tid >> 6) * kColChunk + (tid & 63)] = h;
    __syncthreads();
    if (tid < c - CK.cb) {
      double t = colsh[tid];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) t += colsh[w * kColChunk + tid];
      col_store(a, CK, c0, c1, lw, k0w, k1w, t);
    }
  };
  auto close = [&]() {
    col_park(s, c - CK.cb, h);
    s = 0.0;
    ++c;
    if (c < c1) {
      if (c - CK.cb == kColChunk) {
        flush();
        __syncthreads();   // LDS slots reused by the next chunk
        col_chunk_reload(a, c, CK);
      }
      col_bounds(CK, c, k0w, k1w, lo, hi);
    }
  };
  // distribute one round's products over the columns it meets
  auto consume = [&](const AdjStage<ST>& cur, const float (&gv)[8], int round) {
    const int base = kb + round * kAdjStep, end = base + kAdjStep;
    while (c < c1 && lo < end) {
      if (lo <= base && hi >= end) {
        s += adj_dot(cur, gv);
        if (hi == end) close();
        break;
      }
      s += adj_dot_masked(cur, gv, base + 256 * (tid >> 6) + (tid & 63), lo, hi);
      if (hi > end) break;
      close();
    }
  };
  // round 0 (its gathers and round 1's loads already issued), then the rest
  // alternating between the two register stages
  int round = 0;
  if (nrounds > 0) {
    consume(A, g, 0);
    round = 1;
    auto step = [&](const AdjStage<ST>& cur, AdjStage<ST>& nxt) {
      float gv[8];
      adj_gather(rr, cur, gv);
      // The next round's loads go out after this round's gathers and also
      // past the last round (zeros out of bounds): loads complete in issue
      // order, so either a branch here or loads moved ahead of the gathers
      // would make the wait for the gathers wait for these loads as well.
      __builtin_amdgcn_sched_barrier(0);
      adj_issue<ST, CP>(ri, rv, round + 1, nxt);
      consume(cur, gv, round);
      ++round;
      return round < nrounds;
    };
    while (round < nrounds) {
      if (!step(B, A)) break;
      if (!step(A, B)) break;
    }
  }
  // empty columns at the end of the range
  while (c < c1) close();
  if (c1 > c0) flush();
}

template <int NT, bool SOLVE, int ST, int CP = 0>
__global__ __launch_bounds__(kThreads) void adj_kernel(AdjArgs a) {
  adj_pass<NT, SOLVE, ST, CP>(a, Slot{static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x)});
}

// Batched solve pass (slots as for fwd_wave_batch_kernel).
template <int NT, int ST, int CP = 0>
__global__ __launch_bounds__(kThreads) void adj_batch_kernel(const AdjArgs* __restrict__ args,
                                                             const int32_t* __restrict__ slots) {
  const int sv = uniform(slots[blockIdx.x]);
  if (sv < 0) return;
  // read in place (uniform, read-only): a local copy would live in scratch
  const AdjArgs& a = args[sv >> 16];
  adj_pass<NT, true, ST, CP>(a, Slot{sv & 0xFFFF, a.grid});
}

// Adjoint pass of n <= K solves that share one dose matrix (the same CSC
// arrays and work partition; re-plans of one resident patient): the
// matrix stream of the workgroup's range is read once, and every solve gets
// exactly the arithmetic adj_pass gives it alone -- its own decision, its
// residual gathers, its float64 column sums in the same order and the same
// workgroup-level reductions, its outputs.  plans[q] indexes args.
template <int NT, int ST, int K>
__device__ __forceinline__ void adj_multi_pass(const AdjArgs* __restrict__ args, const int32_t* plans, int n,
                                               const Slot sl) {
  __shared__ double red[kWaves];
  __shared__ double colsh[K][kWaves * kColChunk];
  __shared__ Decision dec[K];
  const AdjArgs& a = args[uniform(plans[0])];   // the shared matrix and partition
  const int tid = threadIdx.x;
  const int lw = logical_wg(sl, a.xcd_map != 0);
  const int k0w = split_point(lw, static_cast<int>(a.nnz), a.grid);
  const int k1w = split_point(lw + 1, static_cast<int>(a.nnz), a.grid);
  const int kb = k0w & ~(kTile - 1);
  const int nrounds = (k1w > kb) ? (k1w - kb + kAdjStep - 1) / kAdjStep : 0;
  const uint32_t bytes = static_cast<uint32_t>((((k1w + kTile - 1) & ~(kTile - 1)) - kb) * 4);
  const rsrc_t ri = make_rsrc(a.row_idx + kb, bytes);
  const rsrc_t rv = (ST == ST_F32) ? make_rsrc(a.val + kb, bytes) : make_rsrc(a.val16 + kb, bytes / 2);
  int pi[K];
#pragma unroll
  for (int q = 0; q < K; ++q) pi[q] = uniform(plans[q < n ? q : 0]);
  DecideLoads<NT> DL[K];
#pragma unroll
  for (int q = 0; q < K; ++q) decide_start<NT>(args[pi[q]], DL[q]);
  const int4 wi = load_i4(make_rsrc(a.wg_cols, 16u * static_cast<uint32_t>(a.grid)), 16u * static_cast<uint32_t>(lw));
  AdjStage<ST> A, B;
  adj_issue(ri, rv, 0, A);
  adj_issue(ri, rv, 1, B);
  const int c0 = uniform(wi.x), c1 = uniform(wi.y);
  int c = c0, lo = uniform(wi.z), hi = uniform(wi.w);
  ColChunk<ST> CK;
  col_chunk_load(a, c0, CK);
  const uint32_t rbytes = 4u * static_cast<uint32_t>(a.nv);
  rsrc_t rr[K];
  float g[K][8];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    rr[q] = make_rsrc(q < n ? args[pi[q]].rbuf[0] : nullptr, q < n ? rbytes : 0u);
    adj_gather(rr[q], A, g[q]);
  }
  bool need[K];
  bool any = false;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    need[q] = false;
    if (q < n) {
      const AdjArgs& aq = args[pi[q]];
      decide<NT>(aq.fwd_partials, aq.fwd_parts, aq.step_partials, aq.step_parts, DL[q], dec[q], red, aq.G_skip);
      if (sl.w == 0 && tid == 0) {
        *aq.st_out = dec[q].st;
        if (dec[q].accepted >= 0 && aq.trace != nullptr && dec[q].st.k - 1 < dec[q].st.trace_cap) {
          TraceDev e;
          e.k = dec[q].st.k;
          e.backtracks = dec[q].backtracks;
          e.lambda = dec[q].lam;
          e.step_sq = dec[q].step_sq;
          e.G = dec[q].st.G;
          aq.trace[dec[q].st.k - 1] = e;
        }
      }
      need[q] = dec[q].st.phase == PH_NEED_GRAD;
      if (need[q] && dec[q].st.acc != 0) {
        rr[q] = make_rsrc(select_buf(aq.rbuf, dec[q].st.acc), rbytes);
        adj_gather(rr[q], A, g[q]);
      }
      if (!need[q]) rr[q] = make_rsrc(nullptr, 0u);
      any = any || need[q];
    }
  }
  if (!any) return;

  double s[K], h[K];
#pragma unroll
  for (int q = 0; q < K; ++q) s[q] = h[q] = 0.0;
  auto flush = [&]() {
#pragma unroll
    for (int q = 0; q < K; ++q)
      if (need[q]) colsh[q][(tid >> 6) * kColChunk + (tid & 63)] = h[q];
    __syncthreads();
    if (tid < c - CK.cb) {
#pragma unroll
      for (int q = 0; q < K; ++q) {
        if (!need[q]) continue;
        double t = colsh[q][tid];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) t += colsh[q][w * kColChunk + tid];
        col_store(args[pi[q]], CK, c0, c1, lw, k0w, k1w, t);
      }
    }
  };
  auto close = [&]() {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      if (!need[q]) continue;
      col_park(s[q], c - CK.cb, h[q]);
      s[q] = 0.0;
    }
    ++c;
    if (c < c1) {
      if (c - CK.cb == kColChunk) {
        flush();
        __syncthreads();   // LDS slots reused by the next chunk
        col_chunk_reload(a, c, CK);
      }
      col_bounds(CK, c, k0w, k1w, lo, hi);
    }
  };
  auto consume = [&](const AdjStage<ST>& cur, const float (&gv)[K][8], int round) {
    const int base = kb + round * kAdjStep, end = base + kAdjStep;
    while (c < c1 && lo < end) {
      if (lo <= base && hi >= end) {
#pragma unroll
        for (int q = 0; q < K; ++q)
          if (need[q]) s[q] += adj_dot(cur, gv[q]);
        if (hi == end) close();
        break;
      }
      const int e0 = base + 256 * (tid >> 6) + (tid & 63);
#pragma unroll
      for (int q = 0; q < K; ++q)
        if (need[q]) s[q] += adj_dot_masked(cur, gv[q], e0, lo, hi);
      if (hi > end) break;
      close();
    }
  };
  int round = 0;
  if (nrounds > 0) {
    consume(A, g, 0);
    round = 1;
    auto step = [&](const AdjStage<ST>& cur, AdjStage<ST>& nxt) {
      float gv[K][8];
#pragma unroll
      for (int q = 0; q < K; ++q) adj_gather(rr[q], cur, gv[q]);
      // The next round's loads go out after this round's gathers and also
      // past the last round (zeros out of bounds): loads complete in issue
      // order, so either a branch here or loads moved ahead of the gathers
      // would make the wait for the gathers wait for these loads as well.
      __builtin_amdgcn_sched_barrier(0);
      adj_issue(ri, rv, round + 1, nxt);
      consume(cur, gv, round);
      ++round;
      return round < nrounds;
    };
    while (round < nrounds) {
      if (!step(B, A)) break;
      if (!step(A, B)) break;
    }
  }
  while (c < c1) close();
  if (c1 > c0) flush();
}

// Batched adjoint pass over groups of solves sharing a dose matrix:
// slots[blockIdx.x] = (group << 16) | workgroup (or -1), groups[(K + 1) g]
// = the group's size n, then its n plan indices.
template <int NT, int ST, int K>
__global__ __launch_bounds__(kThreads) void adj_multi_batch_kernel(const AdjArgs* __restrict__ args,
                                                                   const int32_t* __restrict__ groups,
                                                                   const int32_t* __restrict__ slots) {
  const int sv = uniform(slots[blockIdx.x]);
  if (sv < 0) return;
  const int32_t* gr = groups + static_cast<size_t>(sv >> 16) * (K + 1);
  const int n = uniform(gr[0]);
  adj_multi_pass<NT, ST, K>(args, gr + 1, n, Slot{sv & 0xFFFF, args[uniform(gr[1])].grid});
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
  const double f = (a.col_scale == nullptr) ? a.scale : a.scale * static_cast<double>(a.col_scale[c]);
  a.out[c] = static_cast<float>(f * tot);
}

// ---- small utility kernels ----------------------------------------------------------
__global__ __launch_bounds__(kThreads) void sum_kernel(const double* parts, int n, double* out, double add) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) s += parts[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s + add;
}

__global__ __launch_bounds__(kThreads) void zero_kernel(float* p, int n) {
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) p[i] = 0.0f;
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

__global__ __launch_bounds__(kThreads) void permute_kernel(const float* in, const int32_t* vox, int n, float* out,
                                                           int scatter) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  if (scatter) out[vox[p]] = in[p];
  else out[p] = in[vox[p]];
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

size_t forward_lds_bytes(int nb, int ntrials, int nstruct, bool wave, int storage, int dose_waves) {
  const size_t nbp = static_cast<size_t>(pad4(nb));
  size_t bytes = static_cast<size_t>(nstruct) * sizeof(PenaltyDev) +
                 static_cast<size_t>(ntrials) * nbp * sizeof(float);
  if (wave) {
    const size_t waves = static_cast<size_t>(forward_waves(ntrials, dose_waves));
    bytes += (waves * ntrials * wave_nnz(storage) + kWaveSlack) * sizeof(float);
    bytes += (2 * (kMetaChunk + 1) + kMetaChunk + 2) * sizeof(int32_t) +
             static_cast<size_t>(ntrials) * kMetaChunk * sizeof(double);
  } else {
    bytes += static_cast<size_t>(ntrials) * kFwdNnzMax * sizeof(float) +
             static_cast<size_t>(kFwdRowsMax + 1) * sizeof(int32_t) + kFwdRowsMax;
  }
  return bytes;
}

int forward_waves(int ntrials, int dose_waves) { return (ntrials <= 2 && dose_waves == 16) ? 16 : 8; }

int forward_grid(const imrt_ctx* ctx, const imrt_dose* D, int ntrials) {
  if (ctx->tune.fwd_wave) return wave_grid(ctx, D->nwblocks, ntrials, D->fwd_bpw, D->nb, D->fwd_st, D->fwd_waves);
  return grid_for(D->nblocks, kWaves * ctx->tune.fwd_grid_per_cu * ctx->num_cu);
}

// Forward workgroups per compute unit: the setting, but no more than fit
// side by side -- by registers (one 16-wave workgroup; three 8-wave ones with
// one trial per pass, two with more) and by LDS (the staged vectors grow with
// nb; a structure table of 16 entries assumed) -- since a workgroup that does
// not fit would only start once another has finished.
int wave_grid(const imrt_ctx* ctx, int nwblocks, int ntrials, int blocks_per_wave, int nb, int storage,
              int dose_waves) {
  const int waves = forward_waves(ntrials, dose_waves);
  const int64_t per = static_cast<int64_t>(waves) * std::max(blocks_per_wave, 1);
  const size_t lds = forward_lds_bytes(nb, ntrials, 16, true, storage, dose_waves);
  const int by_lds = static_cast<int>(std::max<size_t>(1, ctx->cu_lds / std::max<size_t>(lds, 1)));
  const int by_regs = (waves == 16) ? 1 : (ntrials == 1) ? 3 : 2;
  const int per_cu = std::max(1, std::min({ctx->tune.fwd_grid_per_cu, by_regs, by_lds}));
  return grid_for(static_cast<int>((nwblocks + per - 1) / per), per_cu * ctx->num_cu);
}

int adjoint_grid_for(const imrt_ctx* ctx, int64_t nnz, int min_nnz) {
  const int64_t cap = static_cast<int64_t>(ctx->tune.adj_grid_per_cu) * ctx->num_cu;
  // at least min_nnz nonzeros per workgroup, at least one workgroup
  const int64_t per = std::max(min_nnz, 1);
  const int64_t want = (nnz + per - 1) / per;
  return static_cast<int>(std::max<int64_t>(1, std::min(cap, want)));
}

// Launches take optional start/stop events, recorded by the dispatch itself
// around the kernel (hipExtLaunchKernelGGL), so their elapsed time is the
// kernel's own duration.
template <int ST, int CP>
int launch_wave_solve(const FwdArgs& a, int ntrials, bool w16, dim3 gd, size_t lds, hipStream_t s, hipEvent_t before,
                      hipEvent_t after) {
  const dim3 bd16(16 * 64), bd8(8 * 64);
  switch (ntrials) {
    case 1:
      if (w16) hipExtLaunchKernelGGL((fwd_wave_kernel<1, FWD_SOLVE, 16, ST, CP>), gd, bd16, lds, s, before, after, 0, a);
      else hipExtLaunchKernelGGL((fwd_wave_kernel<1, FWD_SOLVE, 8, ST, CP>), gd, bd8, lds, s, before, after, 0, a);
      break;
    case 2:
      if (w16) hipExtLaunchKernelGGL((fwd_wave_kernel<2, FWD_SOLVE, 16, ST, CP>), gd, bd16, lds, s, before, after, 0, a);
      else hipExtLaunchKernelGGL((fwd_wave_kernel<2, FWD_SOLVE, 8, ST, CP>), gd, bd8, lds, s, before, after, 0, a);
      break;
    case 4: hipExtLaunchKernelGGL((fwd_wave_kernel<4, FWD_SOLVE, 8, ST, CP>), gd, bd8, lds, s, before, after, 0, a); break;
    default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
  }
  return IMRT_OK;
}

template <int ST>
int launch_wave_forward(const FwdArgs& a, int ntrials, dim3 gd, size_t lds, hipStream_t s, hipEvent_t before,
                        hipEvent_t after) {
  const dim3 bd16(16 * 64), bd8(8 * 64);
  const bool w16 = forward_waves(ntrials, a.waves) == 16;
  if (a.mode == FWD_SOLVE) {
    return a.stream_cp ? launch_wave_solve<ST, 2>(a, ntrials, w16, gd, lds, s, before, after)
                       : launch_wave_solve<ST, 0>(a, ntrials, w16, gd, lds, s, before, after);
  } else if (ntrials != 1) {
    return set_error(IMRT_EINVAL, "evaluation passes take one trial");
  } else if (a.mode == FWD_EVAL) {
    if (w16) hipExtLaunchKernelGGL((fwd_wave_kernel<1, FWD_EVAL, 16, ST>), gd, bd16, lds, s, before, after, 0, a);
    else hipExtLaunchKernelGGL((fwd_wave_kernel<1, FWD_EVAL, 8, ST>), gd, bd8, lds, s, before, after, 0, a);
  } else {
    if (w16) hipExtLaunchKernelGGL((fwd_wave_kernel<1, FWD_PLAIN, 16, ST>), gd, bd16, lds, s, before, after, 0, a);
    else hipExtLaunchKernelGGL((fwd_wave_kernel<1, FWD_PLAIN, 8, ST>), gd, bd8, lds, s, before, after, 0, a);
  }
  return IMRT_OK;
}

// Batched solve passes: one dispatch over the slot table of several plans
// (all with the same storage, forward workgroup size and trials per pass).
template <int ST, int CP>
int launch_forward_batch_st(const FwdArgs* args, const int32_t* slots, int nslots, int ntrials, int dose_waves,
                            size_t lds, hipStream_t s) {
  const dim3 gd(nslots);
  const bool w16 = forward_waves(ntrials, dose_waves) == 16;
  switch (ntrials) {
    case 1:
      if (w16) hipLaunchKernelGGL((fwd_wave_batch_kernel<1, 16, ST, CP>), gd, dim3(16 * 64), lds, s, args, slots);
      else hipLaunchKernelGGL((fwd_wave_batch_kernel<1, 8, ST, CP>), gd, dim3(8 * 64), lds, s, args, slots);
      break;
    case 2:
      if (w16) hipLaunchKernelGGL((fwd_wave_batch_kernel<2, 16, ST, CP>), gd, dim3(16 * 64), lds, s, args, slots);
      else hipLaunchKernelGGL((fwd_wave_batch_kernel<2, 8, ST, CP>), gd, dim3(8 * 64), lds, s, args, slots);
      break;
    case 4: hipLaunchKernelGGL((fwd_wave_batch_kernel<4, 8, ST, CP>), gd, dim3(8 * 64), lds, s, args, slots); break;
    default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
  }
  return IMRT_OK;
}

int launch_forward_batch(const imrt_ctx* ctx, const FwdArgs* args, const int32_t* slots, int nslots, int ntrials,
                         int storage, int dose_waves, size_t lds, int stream_cp) {
  if (nslots <= 0) return IMRT_OK;
  if (lds > ctx->max_lds) return set_error(IMRT_EUNSUPPORTED, "batched forward pass: LDS budget exceeded");
  int rc;
  const int w = dose_waves;
  hipStream_t s = ctx->stream;
  switch (storage) {
    case ST_F32:
      rc = stream_cp ? launch_forward_batch_st<ST_F32, 2>(args, slots, nslots, ntrials, w, lds, s)
                     : launch_forward_batch_st<ST_F32, 0>(args, slots, nslots, ntrials, w, lds, s);
      break;
    case ST_BF16:
      rc = stream_cp ? launch_forward_batch_st<ST_BF16, 2>(args, slots, nslots, ntrials, w, lds, s)
                     : launch_forward_batch_st<ST_BF16, 0>(args, slots, nslots, ntrials, w, lds, s);
      break;
    case ST_F16:
      rc = stream_cp ? launch_forward_batch_st<ST_F16, 2>(args, slots, nslots, ntrials, w, lds, s)
                     : launch_forward_batch_st<ST_F16, 0>(args, slots, nslots, ntrials, w, lds, s);
      break;
    case ST_F32C16:
      rc = stream_cp ? launch_forward_batch_st<ST_F32C16, 2>(args, slots, nslots, ntrials, w, lds, s)
                     : launch_forward_batch_st<ST_F32C16, 0>(args, slots, nslots, ntrials, w, lds, s);
      break;
    default: return set_error(IMRT_EINVAL, "unknown storage");
  }
  if (rc) return rc;
  return check_launch("fwd_wave_batch_kernel");
}

template <int ST, int CP>
int launch_adjoint_batch_st(const AdjArgs* args, const int32_t* slots, int nslots, int ntrials, hipStream_t s) {
  const dim3 gd(nslots), bd(kThreads);
  switch (ntrials) {
    case 1: hipLaunchKernelGGL((adj_batch_kernel<1, ST, CP>), gd, bd, 0, s, args, slots); break;
    case 2: hipLaunchKernelGGL((adj_batch_kernel<2, ST, CP>), gd, bd, 0, s, args, slots); break;
    case 4: hipLaunchKernelGGL((adj_batch_kernel<4, ST, CP>), gd, bd, 0, s, args, slots); break;
    default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
  }
  return IMRT_OK;
}

int launch_adjoint_batch(const imrt_ctx* ctx, const AdjArgs* args, const int32_t* slots, int nslots, int ntrials,
                         int storage, int stream_cp) {
  if (nslots <= 0) return IMRT_OK;
  int rc;
  switch (storage) {
    case ST_F32:
      rc = stream_cp ? launch_adjoint_batch_st<ST_F32, 2>(args, slots, nslots, ntrials, ctx->stream)
                     : launch_adjoint_batch_st<ST_F32, 0>(args, slots, nslots, ntrials, ctx->stream);
      break;
    case ST_BF16:
      rc = stream_cp ? launch_adjoint_batch_st<ST_BF16, 2>(args, slots, nslots, ntrials, ctx->stream)
                     : launch_adjoint_batch_st<ST_BF16, 0>(args, slots, nslots, ntrials, ctx->stream);
      break;
    case ST_F16:
      rc = stream_cp ? launch_adjoint_batch_st<ST_F16, 2>(args, slots, nslots, ntrials, ctx->stream)
                     : launch_adjoint_batch_st<ST_F16, 0>(args, slots, nslots, ntrials, ctx->stream);
      break;
    default: return set_error(IMRT_EINVAL, "unknown storage");
  }
  if (rc) return rc;
  return check_launch("adj_batch_kernel");
}

template <int ST, int K>
int launch_adjoint_multi_st(const AdjArgs* args, const int32_t* groups, const int32_t* slots, int nslots,
                            int ntrials, hipStream_t s) {
  const dim3 gd(nslots), bd(kThreads);
  switch (ntrials) {
    case 1: hipLaunchKernelGGL((adj_multi_batch_kernel<1, ST, K>), gd, bd, 0, s, args, groups, slots); break;
    case 2: hipLaunchKernelGGL((adj_multi_batch_kernel<2, ST, K>), gd, bd, 0, s, args, groups, slots); break;
    case 4: hipLaunchKernelGGL((adj_multi_batch_kernel<4, ST, K>), gd, bd, 0, s, args, groups, slots); break;
    default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
  }
  return IMRT_OK;
}

template <int K>
int launch_adjoint_multi_k(const AdjArgs* args, const int32_t* groups, const int32_t* slots, int nslots,
                           int ntrials, int storage, hipStream_t s) {
  switch (storage) {
    case ST_F32: return launch_adjoint_multi_st<ST_F32, K>(args, groups, slots, nslots, ntrials, s);
    case ST_BF16: return launch_adjoint_multi_st<ST_BF16, K>(args, groups, slots, nslots, ntrials, s);
    case ST_F16: return launch_adjoint_multi_st<ST_F16, K>(args, groups, slots, nslots, ntrials, s);
    default: return set_error(IMRT_EINVAL, "unknown storage");
  }
}

int launch_adjoint_multi_batch(const imrt_ctx* ctx, const AdjArgs* args, const int32_t* groups, int group_k,
                               const int32_t* slots, int nslots, int ntrials, int storage) {
  if (nslots <= 0) return IMRT_OK;
  int rc;
  switch (group_k) {
    case 2: rc = launch_adjoint_multi_k<2>(args, groups, slots, nslots, ntrials, storage, ctx->stream); break;
    case 4: rc = launch_adjoint_multi_k<4>(args, groups, slots, nslots, ntrials, storage, ctx->stream); break;
    default: return set_error(IMRT_EINVAL, "shared-matrix adjoint groups hold 2 or 4 solves");
  }
  if (rc) return rc;
  return check_launch("adj_multi_batch_kernel");
}

int launch_forward(const imrt_ctx* ctx, const imrt_dose* D, const FwdArgs& a, int ntrials, int grid,
                   hipEvent_t before, hipEvent_t after) {
  (void)D;
  clear_stale_error();
  const bool wave = ctx->tune.fwd_wave != 0;
  const size_t lds = forward_lds_bytes(a.nb, ntrials, a.nstruct, wave, a.storage, a.waves);
  if (lds > ctx->max_lds)
    return set_error(IMRT_EUNSUPPORTED, "forward pass: nb * trials exceeds the LDS budget");
  const dim3 gd(grid), bd(kThreads);
  hipStream_t s = ctx->stream;
  if (wave) {
    int rc = IMRT_OK;
    switch (a.storage) {
      case ST_F32: rc = launch_wave_forward<ST_F32>(a, ntrials, gd, lds, s, before, after); break;
      case ST_BF16: rc = launch_wave_forward<ST_BF16>(a, ntrials, gd, lds, s, before, after); break;
      case ST_F16: rc = launch_wave_forward<ST_F16>(a, ntrials, gd, lds, s, before, after); break;
      case ST_F32C16: rc = launch_wave_forward<ST_F32C16>(a, ntrials, gd, lds, s, before, after); break;
      default: return set_error(IMRT_EINVAL, "unknown storage");
    }
    if (rc) return rc;
  } else {
    if (coded(a.storage))   // (ST_F32C16 matrices keep their 32-bit column indices for this pass)
      return set_error(IMRT_EUNSUPPORTED, "16-bit storage needs the wave-granular forward pass (fwd_wave = 1)");
    switch (ntrials) {
      case 1: hipExtLaunchKernelGGL(fwd_kernel<1>, gd, bd, lds, s, before, after, 0, a); break;
      case 2: hipExtLaunchKernelGGL(fwd_kernel<2>, gd, bd, lds, s, before, after, 0, a); break;
      case 4: hipExtLaunchKernelGGL(fwd_kernel<4>, gd, bd, lds, s, before, after, 0, a); break;
      default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
    }
  }
  return check_launch("fwd_kernel");
}

template <int ST, int CP>
int launch_adjoint_kernel(const AdjArgs& a, int ntrials, dim3 gd, dim3 bd, hipStream_t s, hipEvent_t before,
                          hipEvent_t after) {
  switch (a.solve ? ntrials : 0) {
    case 0: hipExtLaunchKernelGGL((adj_kernel<1, false, ST>), gd, bd, 0, s, before, after, 0, a); break;
    case 1: hipExtLaunchKernelGGL((adj_kernel<1, true, ST, CP>), gd, bd, 0, s, before, after, 0, a); break;
    case 2: hipExtLaunchKernelGGL((adj_kernel<2, true, ST, CP>), gd, bd, 0, s, before, after, 0, a); break;
    case 4: hipExtLaunchKernelGGL((adj_kernel<4, true, ST, CP>), gd, bd, 0, s, before, after, 0, a); break;
    default: return set_error(IMRT_EINVAL, "trials per pass must be 1, 2 or 4");
  }
  return IMRT_OK;
}

int launch_adjoint(const imrt_ctx* ctx, const imrt_dose* D, const AdjArgs& a, int ntrials, hipEvent_t before,
                   hipEvent_t after) {
  clear_stale_error();
  const dim3 gd(a.grid), bd(kThreads);
  hipStream_t s = ctx->stream;
  if (!a.solve && ntrials != 1) return set_error(IMRT_EINVAL, "a plain adjoint pass takes one vector");
  int rc = IMRT_OK;
  switch (a.storage) {
    case ST_F32:
      rc = (a.solve && a.stream_cp) ? launch_adjoint_kernel<ST_F32, 2>(a, ntrials, gd, bd, s, before, after)
                                    : launch_adjoint_kernel<ST_F32, 0>(a, ntrials, gd, bd, s, before, after);
      break;
    case ST_BF16:
      rc = (a.solve && a.stream_cp) ? launch_adjoint_kernel<ST_BF16, 2>(a, ntrials, gd, bd, s, before, after)
                                    : launch_adjoint_kernel<ST_BF16, 0>(a, ntrials, gd, bd, s, before, after);
      break;
    case ST_F16:
      rc = (a.solve && a.stream_cp) ? launch_adjoint_kernel<ST_F16, 2>(a, ntrials, gd, bd, s, before, after)
                                    : launch_adjoint_kernel<ST_F16, 0>(a, ntrials, gd, bd, s, before, after);
      break;
    default: return set_error(IMRT_EINVAL, "unknown storage");
  }
  if (rc) return rc;
  rc = check_launch("adj_kernel");
  if (rc) return rc;
  if (!a.solve) {
    // shared columns completed here (in a solve the next forward pass
    // completes them while it stages its trial points)
    const int g2 = (a.nb + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(adj_final_kernel, dim3(g2), dim3(kThreads), 0, s, a, static_cast<const SolverState*>(nullptr));
    rc = check_launch("adj_final_kernel");
  }
  (void)D;
  return rc;
}

int launch_sum(const imrt_ctx* ctx, const double* parts, int n, double* out, double add) {
  clear_stale_error();
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kThreads), 0, ctx->stream, parts, n, out, add);
  return check_launch("sum_kernel");
}

int launch_zero(const imrt_ctx* ctx, float* p, int n) {
  if (n <= 0) return IMRT_OK;
  clear_stale_error();
  const int g = std::min((n + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(zero_kernel, dim3(g), dim3(kThreads), 0, ctx->stream, p, n);
  return check_launch("zero_kernel");
}

int launch_project(const imrt_ctx* ctx, const float* x, const float* g, double lambda, int nb,
                   float* x_out, double* s_out) {
  clear_stale_error();
  hipLaunchKernelGGL(project_kernel, dim3(1), dim3(kThreads), 0, ctx->stream, x, g, lambda, nb, x_out, s_out);
  return check_launch("project_kernel");
}

int launch_permute(const imrt_ctx* ctx, const float* in, const int32_t* vox, int n, float* out, bool scatter) {
  clear_stale_error();
  hipLaunchKernelGGL(permute_kernel, dim3(grid_for((n + kThreads - 1) / kThreads, 1 << 30)), dim3(kThreads), 0,
                     ctx->stream, in, vox, n, out, scatter ? 1 : 0);
  return check_launch("permute_kernel");
}

int launch_normalize(const imrt_ctx* ctx, const float* w, int nb, float* v_out, double* norm_out) {
  clear_stale_error();
  hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(kThreads), 0, ctx->stream, w, nb, v_out, norm_out);
  return check_launch("normalize_kernel");
}

}  // namespace imrt
