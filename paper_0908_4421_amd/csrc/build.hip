// Synthetic prostate-shaped phantom and its dose-deposition matrix D, built on
// the device.  D plays the role of the dose deposition coefficients of
// Section 2.1 (dose to voxel j from beamlet i at unit intensity); the paper
// takes it from a clinical dose engine, here a pencil-beam model stands in.
//
// Every float64 expression is evaluated in one fixed order with contraction
// off (this file is compiled with -ffp-contract=off as well), so the sparsity
// pattern is a deterministic function of the geometry:
//   voxel centre   p_a = (i_a + 0.5)*h - (n_a*h)/2
//   depth          -max over in-plane axes with dir_a != 0 of
//                  min((lo_a - p_a)/dir_a, (hi_a - p_a)/dir_a)
//   lateral        u = (-sin)*x + cos*y,  v = z
//   exponent       e = (mu*depth) + (((u-u_c)^2 + (v-v_c)^2) / ((2*sigma)*sigma))
//   kept           e <= e_min(beamlet) + log(1/tau), e_min over every grid voxel
//   value          float32(exp(-e))
// Beam angles' cosines/sines and log(1/tau) are computed once on the host.
//
// Unspecified tissue at twice the voxel size (Section 3.1): with
// coarse_normal, every aligned, complete 2x2x2 block of grid voxels that are
// all normal tissue becomes one voxel centred at
//   c_a = (2*b_a + 1)*h - (n_a*h)/2
// of structure "normal".  The voxels crossing the API are then the remaining
// grid voxels (grid index ascending) followed by the coarse voxels (block
// index bx + (nx/2)*(by + (ny/2)*bz) ascending).
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <vector>

#include "imrt_internal.h"

namespace imrt {
namespace {

struct Geo {
  int nx, ny, nz;
  int ngrid, nv;               // grid voxels; rows of D (the layout's voxels)
  int cx, cy;                  // coarse blocks per x row and per y column (nx/2, ny/2)
  double h, hx, hy;            // half extents (n*h)/2 in x and y
  double r_ptv, r_rectum, r_bladder;
  double mu, two_sig2;         // (2*sigma)*sigma
  double keep_log;             // log(1/tau)
  int nbeam;
};

struct BeamletDev {
  int32_t beam;
  int32_t pad;
  double u_c, v_c;
};

__device__ __forceinline__ double centre(int i, int n, double h) {
  return (static_cast<double>(i) + 0.5) * h - (static_cast<double>(n) * h) / 2.0;
}

__device__ __forceinline__ void voxel_xyz(const Geo& g, int j, double& x, double& y, double& z) {
  const int ix = j % g.nx;
  const int t = j / g.nx;
  const int iy = t % g.ny;
  const int iz = t / g.ny;
  x = centre(ix, g.nx, g.h);
  y = centre(iy, g.ny, g.h);
  z = centre(iz, g.nz, g.h);
}

__device__ __forceinline__ double coarse_centre(int b, int n, double h) {
  return (2.0 * static_cast<double>(b) + 1.0) * h - (static_cast<double>(n) * h) / 2.0;
}

// Centre of the voxel with point code c: a grid index (c >= 0) or the coarse
// block -1 - c.
__device__ __forceinline__ void voxel_point(const Geo& g, int c, double& x, double& y, double& z) {
  if (c >= 0) {
    voxel_xyz(g, c, x, y, z);
    return;
  }
  const int b = -1 - c;
  const int bx = b % g.cx;
  const int t = b / g.cx;
  x = coarse_centre(bx, g.nx, g.h);
  y = coarse_centre(t % g.cy, g.ny, g.h);
  z = coarse_centre(t / g.cy, g.nz, g.h);
}

__device__ __forceinline__ void depth_u(const Geo& g, double x, double y, double c, double s,
                                        double& depth, double& u) {
  double t = 0.0;
  bool have = false;
  if (c != 0.0) {
    t = fmin((-g.hx - x) / c, (g.hx - x) / c);
    have = true;
  }
  if (s != 0.0) {
    const double ty = fmin((-g.hy - y) / s, (g.hy - y) / s);
    t = have ? fmax(t, ty) : ty;
  }
  depth = -t;
  u = (-s) * x + c * y;
}

__device__ __forceinline__ double exponent(const Geo& g, double depth, double u, double z,
                                           double uc, double vc) {
  const double du = u - uc;
  const double dv = z - vc;
  const double r2 = du * du + dv * dv;
  return (g.mu * depth) + (r2 / g.two_sig2);
}

// Rows of D follow the internal voxel order: row p is the voxel with point
// code code[p] (grid voxel p itself when code is NULL).
__device__ __forceinline__ int code_of(const int32_t* code, int p) { return code ? code[p] : p; }

// Structure id of rows [0, n): coarse voxels are normal tissue.
__global__ __launch_bounds__(kThreads) void structure_kernel(Geo g, int n, const int32_t* code, uint8_t* sid) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const int c = code_of(code, p);
  if (c < 0) {
    sid[p] = 0;
    return;
  }
  double x, y, z;
  voxel_xyz(g, c, x, y, z);
  uint8_t s = 0;
  const double cb = g.r_ptv + g.r_bladder;
  const double dyb = y - cb;
  if ((x * x + dyb * dyb) + z * z <= g.r_bladder * g.r_bladder) s = 3;
  const double cr = -(g.r_ptv + g.r_rectum);
  const double dyr = y - cr;
  if (x * x + dyr * dyr <= g.r_rectum * g.r_rectum) s = 2;
  if ((x * x + y * y) + z * z <= g.r_ptv * g.r_ptv) s = 1;
  sid[p] = s;
}

// One workgroup per beamlet: minimum exponent over all voxels (exact; order-free).
__global__ __launch_bounds__(kThreads) void emin_kernel(Geo g, const BeamletDev* bl, const double2* dirs,
                                                        double* emin) {
  const int i = blockIdx.x;
  const BeamletDev b = bl[i];
  const double2 d = dirs[b.beam];
  double m = INFINITY;
  for (int j = threadIdx.x; j < g.ngrid; j += kThreads) {
    double x, y, z, depth, u;
    voxel_xyz(g, j, x, y, z);
    depth_u(g, x, y, d.x, d.y, depth, u);
    m = fmin(m, exponent(g, depth, u, z, b.u_c, b.v_c));
  }
  __shared__ double sh[kThreads];
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) emin[i] = sh[0];
}

// One workgroup per beamlet: ordered compaction of the kept voxels (CSC).
// With fill == false only the count is produced.
__global__ __launch_bounds__(kThreads) void column_kernel(Geo g, const int32_t* code, const BeamletDev* bl,
                                                          const double2* dirs, const double* emin, int32_t* counts,
                                                          const int32_t* col_ptr, int32_t* row_idx,
                                                          float* cval, int fill) {
  const int i = blockIdx.x;
  const BeamletDev b = bl[i];
  const double2 d = dirs[b.beam];
  const double limit = emin[i] + g.keep_log;
  const int nv = g.nv;
  __shared__ int wave_cnt[kWaves];
  __shared__ int base;
  if (threadIdx.x == 0) base = fill ? col_ptr[i] : 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int p0 = 0; p0 < nv; p0 += kThreads) {
    const int p = p0 + threadIdx.x;
    bool keep = false;
    double e = 0.0;
    if (p < nv) {
      double x, y, z, depth, u;
      voxel_point(g, code_of(code, p), x, y, z);
      depth_u(g, x, y, d.x, d.y, depth, u);
      e = exponent(g, depth, u, z, b.u_c, b.v_c);
      keep = e <= limit;
    }
    const unsigned long long mask = __ballot(keep);
    if (lane == 0) wave_cnt[w] = __popcll(mask);
    __syncthreads();
    int before = base;
    for (int k = 0; k < w; ++k) before += wave_cnt[k];
    if (keep && fill) {
      const int64_t pos = csc_slot(before + __popcll(mask & ((1ull << lane) - 1ull)));
      row_idx[pos] = p;
      cval[pos] = static_cast<float>(exp(-e));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int k = 0; k < kWaves; ++k) tot += wave_cnt[k];
      base += tot;
    }
    __syncthreads();
  }
  if (!fill && threadIdx.x == 0) counts[i] = base;
}

// One thread per voxel: kept beamlets in ascending column order (CSR).
__global__ __launch_bounds__(kThreads) void row_kernel(Geo g, const int32_t* code, const BeamletDev* bl,
                                                       const int32_t* beam_first, const double2* dirs,
                                                       const double* emin, int32_t* counts, const int32_t* row_ptr,
                                                       int32_t* col_idx, float* val, int fill) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= g.nv) return;
  double x, y, z;
  voxel_point(g, code_of(code, p), x, y, z);
  int pos = fill ? row_ptr[p] : 0;
  for (int beam = 0; beam < g.nbeam; ++beam) {
    const double2 d = dirs[beam];
    double depth, u;
    depth_u(g, x, y, d.x, d.y, depth, u);
    for (int i = beam_first[beam]; i < beam_first[beam + 1]; ++i) {
      const double e = exponent(g, depth, u, z, bl[i].u_c, bl[i].v_c);
      if (e <= emin[i] + g.keep_log) {
        if (fill) {
          col_idx[pos] = i;
          val[pos] = static_cast<float>(exp(-e));
        }
        ++pos;
      }
    }
  }
  if (!fill) counts[p] = pos;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// ---- 16-bit storage ---------------------------------------------------------------
// Code of a nonnegative float64 quotient v = D_ij / s_i in bfloat16 (8
// significand bits, smallest normal exponent -126) or binary16 (11, -14):
// with 2^e <= v < 2^(e+1), the quantum is 2^(max(e, emin) - p + 1); v divided
// by it is exact, rint rounds it to nearest with ties to even, and the rounded
// value is representable in float32 and in the 16-bit format.  The float64
// quotient of two float32 numbers never lands on (or across) a tie of these
// formats unless the exact quotient does, so this is the rounding of the
// exact quotient.
template <int ST>
__device__ uint16_t code16(double v) {
  if (!(v > 0.0)) return 0;
  constexpr int p = (ST == ST_BF16) ? 8 : 11;
  constexpr int emin = (ST == ST_BF16) ? -126 : -14;
  int E = 0;
  (void)frexp(v, &E);   // v = m 2^E, 1/2 <= m < 1
  const int qe = max(E - 1, emin) - (p - 1);
  const float f = static_cast<float>(ldexp(rint(ldexp(v, -qe)), qe));
  if (ST == ST_BF16) return static_cast<uint16_t>(__float_as_uint(f) >> 16);
  return __builtin_bit_cast(uint16_t, static_cast<_Float16>(f));
}

// One wave per column: s = the largest value (1 when none is positive), then
// the codes of the column's entries in CSC slot order.
template <int ST>
__global__ __launch_bounds__(kThreads) void quantize_columns_kernel(const int32_t* col_ptr, const float* cval,
                                                                     int nb, float* scale, uint16_t* cval16) {
  const int c = blockIdx.x * kWaves + static_cast<int>(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nb) return;
  const int k0 = col_ptr[c], k1 = col_ptr[c + 1];
  float m = 0.0f;
  for (int k = k0 + lane; k < k1; k += 64) m = fmaxf(m, cval[csc_slot(k)]);
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  const float sc = (m > 0.0f) ? m : 1.0f;
  if (lane == 0) scale[c] = sc;
  for (int k = k0 + lane; k < k1; k += 64) {
    const int64_t slot = csc_slot(k);
    cval16[slot] = code16<ST>(static_cast<double>(cval[slot]) / static_cast<double>(sc));
  }
}

// CSR codes and 16-bit column indices.
template <int ST>
__global__ __launch_bounds__(kThreads) void quantize_rows_kernel(const int32_t* col_idx, const float* val, int64_t nnz,
                                                                  const float* scale, uint16_t* col16,
                                                                  uint16_t* val16) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; k < nnz;
       k += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int c = col_idx[k];
    col16[k] = static_cast<uint16_t>(c);
    val16[k] = code16<ST>(static_cast<double>(val[k]) / static_cast<double>(scale[c]));
  }
}

__global__ __launch_bounds__(kThreads) void narrow_columns_kernel(const int32_t* col_idx, int64_t nnz,
                                                                   uint16_t* col16) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; k < nnz;
       k += static_cast<int64_t>(gridDim.x) * kThreads)
    col16[k] = static_cast<uint16_t>(col_idx[k]);
}

// float32 storage read by the forward pass through 16-bit column indices
// (nb <= 65536): a 16-bit copy of the CSR column indices beside the 32-bit
// ones, which the other passes and the export keep using.
int narrow_columns(imrt_dose* D) {
  const size_t nz = static_cast<size_t>(D->nnz) + kPad;
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(&D->col16), 2 * nz);
  if (e == hipErrorOutOfMemory) return set_error(IMRT_ENOMEM, "hipMalloc: out of device memory");
  if (e != hipSuccess) return hip_error(e, "hipMalloc(16-bit column indices)");
  hipStream_t s = D->ctx->stream;
  IMRT_HIP(hipMemsetAsync(D->col16, 0, 2 * nz, s));
  const int gr = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((D->nnz + kThreads - 1) / kThreads, 8192)));
  hipLaunchKernelGGL(narrow_columns_kernel, dim3(gr), dim3(kThreads), 0, s, D->col_idx, D->nnz, D->col16);
  IMRT_HIP(hipGetLastError());
  IMRT_HIP(hipStreamSynchronize(s));
  return IMRT_OK;
}

}  // namespace

int store16(imrt_dose* D, int storage) {
  if (storage == ST_F32) return D->fwd_st == ST_F32C16 ? narrow_columns(D) : IMRT_OK;
  if (storage != ST_BF16 && storage != ST_F16) return set_error(IMRT_EINVAL, "unknown storage");
  if (D->nb > 65536) return set_error(IMRT_EUNSUPPORTED, "16-bit storage needs nb <= 65536 (16-bit column indices)");
  const size_t nz = static_cast<size_t>(D->nnz) + kPad, nzc = csc_alloc(D->nnz);
  auto alloc = [](void** p, size_t bytes) -> int {
    const hipError_t e = hipMalloc(p, bytes < 1 ? 1 : bytes);
    if (e == hipErrorOutOfMemory) return set_error(IMRT_ENOMEM, "hipMalloc: out of device memory");
    if (e != hipSuccess) return hip_error(e, "hipMalloc(16-bit storage)");
    return IMRT_OK;
  };
  int rc;
  if ((rc = alloc(reinterpret_cast<void**>(&D->col_scale), sizeof(float) * std::max(D->nb, 1))) ||
      (rc = alloc(reinterpret_cast<void**>(&D->col16), 2 * nz)) ||
      (rc = alloc(reinterpret_cast<void**>(&D->val16), 2 * nz)) ||
      (rc = alloc(reinterpret_cast<void**>(&D->cval16), 2 * nzc)))
    return rc;
  hipStream_t s = D->ctx->stream;
  IMRT_HIP(hipMemsetAsync(D->col16, 0, 2 * nz, s));
  IMRT_HIP(hipMemsetAsync(D->val16, 0, 2 * nz, s));
  IMRT_HIP(hipMemsetAsync(D->cval16, 0, 2 * nzc, s));
  const int gc = std::max(1, (D->nb + kWaves - 1) / kWaves);
  const int gr = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((D->nnz + kThreads - 1) / kThreads, 8192)));
  if (storage == ST_BF16) {
    hipLaunchKernelGGL(quantize_columns_kernel<ST_BF16>, dim3(gc), dim3(kThreads), 0, s, D->col_ptr, D->cval, D->nb,
                       D->col_scale, D->cval16);
    hipLaunchKernelGGL(quantize_rows_kernel<ST_BF16>, dim3(gr), dim3(kThreads), 0, s, D->col_idx, D->val, D->nnz,
                       D->col_scale, D->col16, D->val16);
  } else {
    hipLaunchKernelGGL(quantize_columns_kernel<ST_F16>, dim3(gc), dim3(kThreads), 0, s, D->col_ptr, D->cval, D->nb,
                       D->col_scale, D->cval16);
    hipLaunchKernelGGL(quantize_rows_kernel<ST_F16>, dim3(gr), dim3(kThreads), 0, s, D->col_idx, D->val, D->nnz,
                       D->col_scale, D->col16, D->val16);
  }
  IMRT_HIP(hipGetLastError());
  IMRT_HIP(hipStreamSynchronize(s));
  // the float32 values and indices are not kept
  IMRT_HIP(hipFree(D->col_idx));
  IMRT_HIP(hipFree(D->val));
  IMRT_HIP(hipFree(D->cval));
  D->col_idx = nullptr;
  D->val = nullptr;
  D->cval = nullptr;
  D->storage = storage;
  return IMRT_OK;
}

int build_phantom(imrt_ctx* ctx, const imrt_geometry* G, imrt_dose* D) {
  if (G->nx <= 0 || G->ny <= 0 || G->nz <= 0 || G->n_beams <= 0)
    return set_error(IMRT_EINVAL, "geometry: grid sizes and beam count must be positive");
  const int64_t nv64 = static_cast<int64_t>(G->nx) * G->ny * G->nz;
  if (nv64 >= (int64_t(1) << 31)) return set_error(IMRT_EINVAL, "geometry: too many voxels");
  if (!(G->h > 0) || !(G->beamlet > 0) || !(G->sigma > 0) || !(G->tau > 0 && G->tau <= 1) ||
      !(G->mu >= 0) || !(G->r_ptv > 0) || !(G->r_rectum >= 0) || !(G->r_bladder >= 0) || !(G->margin >= 0))
    return set_error(IMRT_EINVAL, "geometry: lengths, sigma, tau or mu out of range");
  if (G->coarse_normal != 0 && G->coarse_normal != 1) return set_error(IMRT_EINVAL, "geometry: coarse_normal must be 0 or 1");
  const int ngrid = static_cast<int>(nv64);

  // Beam directions and beamlets on the host (libm cos/sin, exact integer scans).
  std::vector<double2> dirs(G->n_beams);
  for (int b = 0; b < G->n_beams; ++b) {
    const double theta = (2.0 * M_PI * b) / G->n_beams;
    dirs[b] = make_double2(std::cos(theta), std::sin(theta));
  }
  const double w = G->beamlet;
  const double reach = G->r_ptv + G->margin;
  const int kmax = static_cast<int>(std::ceil(reach / w)) + 1;
  std::vector<BeamletDev> bls;
  std::vector<int32_t> beam_first(G->n_beams + 1, 0);
  for (int b = 0; b < G->n_beams; ++b) {
    beam_first[b] = static_cast<int32_t>(bls.size());
    for (int m = -kmax; m < kmax; ++m) {
      const double lo_u = m * w, hi_u = (m + 1) * w;
      const double cu = std::min(std::max(0.0, lo_u), hi_u);
      for (int n = -kmax; n < kmax; ++n) {
        const double lo_v = n * w, hi_v = (n + 1) * w;
        const double cv = std::min(std::max(0.0, lo_v), hi_v);
        if (cu * cu + cv * cv <= reach * reach) bls.push_back({b, 0, (m + 0.5) * w, (n + 0.5) * w});
      }
    }
  }
  beam_first[G->n_beams] = static_cast<int32_t>(bls.size());
  const int nb = static_cast<int>(bls.size());
  if (nb == 0) return set_error(IMRT_EINVAL, "geometry: no beamlets");

  Geo g;
  g.nx = G->nx; g.ny = G->ny; g.nz = G->nz;
  g.ngrid = ngrid;
  g.nv = ngrid;
  g.cx = G->nx / 2;
  g.cy = G->ny / 2;
  g.h = G->h;
  g.hx = (static_cast<double>(G->nx) * G->h) / 2.0;
  g.hy = (static_cast<double>(G->ny) * G->h) / 2.0;
  g.r_ptv = G->r_ptv; g.r_rectum = G->r_rectum; g.r_bladder = G->r_bladder;
  g.mu = G->mu;
  g.two_sig2 = (2.0 * G->sigma) * G->sigma;
  g.keep_log = std::log(1.0 / G->tau);
  g.nbeam = G->n_beams;

  hipStream_t s = ctx->stream;
  (void)hipGetLastError();  // drop an error left by an unrelated earlier call
  DevBuf d_bl, d_first, d_dirs, d_emin, d_cnt_c, d_cnt_r, d_code;
  IMRT_HIP(hipMalloc(&d_bl.p, sizeof(BeamletDev) * nb));
  IMRT_HIP(hipMalloc(&d_first.p, sizeof(int32_t) * (G->n_beams + 1)));
  IMRT_HIP(hipMalloc(&d_dirs.p, sizeof(double2) * G->n_beams));
  IMRT_HIP(hipMalloc(&d_emin.p, sizeof(double) * nb));
  IMRT_HIP(hipMalloc(&d_cnt_c.p, sizeof(int32_t) * nb));
  IMRT_HIP(hipMemcpyAsync(d_bl.p, bls.data(), sizeof(BeamletDev) * nb, hipMemcpyHostToDevice, s));
  IMRT_HIP(hipMemcpyAsync(d_first.p, beam_first.data(), sizeof(int32_t) * (G->n_beams + 1),
                          hipMemcpyHostToDevice, s));
  IMRT_HIP(hipMemcpyAsync(d_dirs.p, dirs.data(), sizeof(double2) * G->n_beams, hipMemcpyHostToDevice, s));

  // Voxel layout.  api_code[a] is the point code of the voxel with API index
  // a (empty for a uniform grid, where the API index is the grid index);
  // fine_api and block_api give the API index of a grid voxel and of a
  // coarse block (-1: merged into a block, or not coarse).
  std::vector<int32_t> api_code, fine_api, block_api;
  int nv = ngrid;
  if (G->coarse_normal) {
    DevBuf d_gsid;
    IMRT_HIP(hipMalloc(&d_gsid.p, static_cast<size_t>(ngrid)));
    hipLaunchKernelGGL(structure_kernel, dim3((ngrid + kThreads - 1) / kThreads), dim3(kThreads), 0, s, g, ngrid,
                       static_cast<const int32_t*>(nullptr), static_cast<uint8_t*>(d_gsid.p));
    IMRT_HIP(hipGetLastError());
    std::vector<uint8_t> gsid(static_cast<size_t>(ngrid));
    IMRT_HIP(hipMemcpyAsync(gsid.data(), d_gsid.p, static_cast<size_t>(ngrid), hipMemcpyDeviceToHost, s));
    IMRT_HIP(hipStreamSynchronize(s));
    const int cx = g.cx, cy = g.cy, cz = G->nz / 2;
    std::vector<uint8_t> merged(static_cast<size_t>(ngrid), 0);
    std::vector<int32_t> blocks;
    block_api.assign(static_cast<size_t>(cx) * cy * cz, -1);
    for (int bz = 0; bz < cz; ++bz)
      for (int by = 0; by < cy; ++by)
        for (int bx = 0; bx < cx; ++bx) {
          bool normal = true;
          for (int d = 0; d < 8 && normal; ++d) {
            const int j = (2 * bx + (d & 1)) + G->nx * ((2 * by + ((d >> 1) & 1)) + G->ny * (2 * bz + (d >> 2)));
            normal = gsid[j] == 0;
          }
          if (!normal) continue;
          blocks.push_back(bx + cx * (by + cy * bz));
          for (int d = 0; d < 8; ++d)
            merged[(2 * bx + (d & 1)) + G->nx * ((2 * by + ((d >> 1) & 1)) + G->ny * (2 * bz + (d >> 2)))] = 1;
        }
    fine_api.assign(static_cast<size_t>(ngrid), -1);
    api_code.reserve(static_cast<size_t>(ngrid));
    for (int j = 0; j < ngrid; ++j)
      if (!merged[j]) {
        fine_api[j] = static_cast<int32_t>(api_code.size());
        api_code.push_back(j);
      }
    for (int32_t b : blocks) {
      block_api[b] = static_cast<int32_t>(api_code.size());
      api_code.push_back(-1 - b);
    }
    nv = static_cast<int>(api_code.size());
  }
  g.nv = nv;

  // Internal voxel order: tiles of 4 x 4 x 2 grid voxels (x fastest inside a
  // tile, tiles in x, y, z order; a tile's coarse voxels after its grid
  // voxels), so that the voxels a beamlet crosses sit close together in
  // memory whatever the beam direction.  Row p of D is the voxel with API
  // index vox[p] and point code codes[p].
  std::vector<int32_t> codes;
  if (ctx->tune.voxel_tiles) {
    constexpr int tx = 4, ty = 4, tz = 2;
    D->vox_host.resize(static_cast<size_t>(nv));
    codes.resize(static_cast<size_t>(nv));
    int64_t p = 0;
    for (int z0 = 0; z0 < G->nz; z0 += tz)
      for (int y0 = 0; y0 < G->ny; y0 += ty)
        for (int x0 = 0; x0 < G->nx; x0 += tx) {
          for (int z = z0; z < std::min(z0 + tz, G->nz); ++z)
            for (int y = y0; y < std::min(y0 + ty, G->ny); ++y)
              for (int x = x0; x < std::min(x0 + tx, G->nx); ++x) {
                const int j = x + G->nx * (y + G->ny * z);
                const int a = api_code.empty() ? j : fine_api[j];
                if (a < 0) continue;
                if (p >= nv) return set_error(IMRT_EINVAL, "internal: voxel tiles overrun the layout");
                D->vox_host[p] = a;
                codes[p] = j;
                ++p;
              }
          if (api_code.empty()) continue;
          const int bz = z0 / 2;
          if (bz >= G->nz / 2) continue;
          for (int by = y0 / 2; by < std::min(y0 / 2 + ty / 2, g.cy); ++by)
            for (int bx = x0 / 2; bx < std::min(x0 / 2 + tx / 2, g.cx); ++bx) {
              const int b = bx + g.cx * (by + g.cy * bz);
              const int a = block_api[b];
              if (a < 0) continue;
              if (p >= nv) return set_error(IMRT_EINVAL, "internal: voxel tiles overrun the layout");
              D->vox_host[p] = a;
              codes[p] = -1 - b;
              ++p;
            }
        }
    if (p != nv) return set_error(IMRT_EINVAL, "internal: voxel tiles do not cover the layout");
    IMRT_HIP(hipMalloc(&D->vox, sizeof(int32_t) * nv));
    IMRT_HIP(hipMemcpyAsync(D->vox, D->vox_host.data(), sizeof(int32_t) * nv, hipMemcpyHostToDevice, s));
  } else if (!api_code.empty()) {
    codes = api_code;   // rows in API order
  }
  if (!codes.empty()) {
    IMRT_HIP(hipMalloc(&d_code.p, sizeof(int32_t) * nv));
    IMRT_HIP(hipMemcpyAsync(d_code.p, codes.data(), sizeof(int32_t) * nv, hipMemcpyHostToDevice, s));
  }
  const int32_t* code = static_cast<const int32_t*>(d_code.p);
  IMRT_HIP(hipMalloc(&d_cnt_r.p, sizeof(int32_t) * nv));
  IMRT_HIP(hipMalloc(&D->sid, nv));
  const int vgrid = (nv + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(structure_kernel, dim3(vgrid), dim3(kThreads), 0, s, g, nv, code, D->sid);
  IMRT_HIP(hipGetLastError());
  const auto* blp = static_cast<const BeamletDev*>(d_bl.p);
  const auto* dp = static_cast<const double2*>(d_dirs.p);
  auto* em = static_cast<double*>(d_emin.p);
  hipLaunchKernelGGL(emin_kernel, dim3(nb), dim3(kThreads), 0, s, g, blp, dp, em);
  IMRT_HIP(hipGetLastError());
  hipLaunchKernelGGL(column_kernel, dim3(nb), dim3(kThreads), 0, s, g, code, blp, dp, em,
                     static_cast<int32_t*>(d_cnt_c.p), nullptr, nullptr, nullptr, 0);
  IMRT_HIP(hipGetLastError());
  hipLaunchKernelGGL(row_kernel, dim3(vgrid), dim3(kThreads), 0, s, g, code, blp,
                     static_cast<const int32_t*>(d_first.p), dp, em, static_cast<int32_t*>(d_cnt_r.p),
                     nullptr, nullptr, nullptr, 0);
  IMRT_HIP(hipGetLastError());

  std::vector<int32_t> ccount(nb), rcount(nv);
  IMRT_HIP(hipMemcpyAsync(ccount.data(), d_cnt_c.p, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
  IMRT_HIP(hipMemcpyAsync(rcount.data(), d_cnt_r.p, sizeof(int32_t) * nv, hipMemcpyDeviceToHost, s));
  IMRT_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> col_ptr(nb + 1, 0), row_ptr(nv + 1, 0);
  int64_t tot_c = 0, tot_r = 0;
  for (int i = 0; i < nb; ++i) {
    tot_c += ccount[i];
    if (tot_c >= (int64_t(1) << 31)) return set_error(IMRT_EUNSUPPORTED, "D has 2^31 or more nonzeros");
    col_ptr[i + 1] = static_cast<int32_t>(tot_c);
  }
  for (int j = 0; j < nv; ++j) {
    tot_r += rcount[j];
    if (tot_r >= (int64_t(1) << 31)) return set_error(IMRT_EUNSUPPORTED, "D has 2^31 or more nonzeros");
    row_ptr[j + 1] = static_cast<int32_t>(tot_r);
  }
  if (tot_c != tot_r) return set_error(IMRT_EINVAL, "internal: CSR and CSC nonzero counts differ");

  D->nv = nv;
  D->nb = nb;
  D->nnz = tot_r;
  const size_t nz = static_cast<size_t>(tot_r);
  (void)nz;
  const int arc = alloc_nonzeros(D);
  if (arc) return arc;
  IMRT_HIP(hipMemcpyAsync(D->row_ptr, row_ptr.data(), sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice, s));
  IMRT_HIP(hipMemcpyAsync(D->col_ptr, col_ptr.data(), sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(column_kernel, dim3(nb), dim3(kThreads), 0, s, g, code, blp, dp, em, nullptr, D->col_ptr,
                     D->row_idx, D->cval, 1);
  IMRT_HIP(hipGetLastError());
  hipLaunchKernelGGL(row_kernel, dim3(vgrid), dim3(kThreads), 0, s, g, code, blp,
                     static_cast<const int32_t*>(d_first.p), dp, em, nullptr, D->row_ptr, D->col_idx,
                     D->val, 1);
  IMRT_HIP(hipGetLastError());
  IMRT_HIP(hipStreamSynchronize(s));
  apply_partition_targets(ctx, D);
  return finish_dose(D, row_ptr, col_ptr);
}

}  // namespace imrt
