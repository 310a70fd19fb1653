// HIP kernels for gfx950: initialisation, observables and density
// extraction, and the dispatch of the step kernels (lbm_step.h, instantiated
// per collision operator in lbm_step_{srt,mrt,trt}.hip).
#include <hip/hip_runtime.h>

#include "lbm_step.h"

namespace lbm {

// ---------------------------------------------------------------------------
// initial state: f*_i = w_i rho0 at fluid nodes (rest equilibrium), and the
// ghost slots of solid sources (FP32 storage).  With a saturation field
// (sat != NULL) the densities are (major, minor) where sat > thr and
// (minor, major) elsewhere instead of rho0.
// ---------------------------------------------------------------------------
template <int Q, int ST>
__global__ void init_kernel(const InstDev *__restrict__ insts, const float *__restrict__ rho0, int parity,
                            const float *__restrict__ sat = nullptr, float thr = 0.f, float major = 0.f,
                            float minor = 0.f) {
  const InstDev &d = insts[0];
  const int64_t n_nodes = (int64_t)d.nx * d.ny * d.nz;
  gf *b = G(d.f[parity]);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < n_nodes;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int x = n % d.nx;
    const int64_t yz = n / d.nx;
    const int y = yz % d.ny, z = yz / d.ny;
    const uint32_t info = d.info[x + (int64_t)d.pitch * yz];
    if (info & kSolid) continue;
    const bool nw = sat && sat[n] > thr;
    const float r1 = sat ? (nw ? major : minor) : rho0[n], r2 = sat ? (nw ? minor : major) : rho0[n_nodes + n];
    float a[Q], c[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      a[i] = (float)(Lat<Q>::w[i] * (double)r1);
      c[i] = (float)(Lat<Q>::w[i] * (double)r2);
    }
    if (d.compact) {
      cpop_store<Q, ST>(b, d.cpitch, crank(d, x, y + (int64_t)d.ny * z), a, c, r1, r2);
      continue;
    }
    pop_store<Q, ST>(b, d.pitch, y * d.ystride + z * d.zstride, x, a, c, r1, r2);
    int64_t src[3][3];
    int xs[3];
    source_rows<Q>(d, y, z, src);
    source_x(d, x, xs);
    store_ghosts<Q, ST>(d, b, info, src, xs, a, c);
  }
}

// ---------------------------------------------------------------------------
// observables: per-block FP64 partial sums in a fixed order
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int Q, int ST>
__global__ __launch_bounds__(256) void obs_kernel(const InstDev *__restrict__ insts, int parity,
                                                  double *__restrict__ partials) {
  const InstDev &d = insts[0];
  gcf *fin = G(d.f[parity]);
  const int64_t n_nodes = (int64_t)d.nx * d.ny * d.nz;
  double acc[kObsFields - 1] = {0};
  int flags = 0;
  const double third = 1.0 / 3.0;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < n_nodes;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int x = n % d.nx;
    const int64_t yz = n / d.nx;
    const int y = yz % d.ny, z = yz / d.ny;
    const uint32_t inf = d.info[x + (int64_t)d.pitch * yz];
    if (inf & kSolid) continue;
    float a[Q], b[Q];
    if (d.compact) cgather<Q, ST, double>(d, fin, inf, x, y, z, crank(d, x, yz), a, b);
    else gather<Q, ST, double>(d, fin, inf, x, y, z, a, b);
    const double r1 = sum_q<Q, double>(a), r2 = sum_q<Q, double>(b);
    if (!isfinite(r1) || !isfinite(r2)) flags |= 1;
    if (r1 < 0.0 || r2 < 0.0) flags |= 2;
    acc[0] += r1;
    acc[1] += r2;
    acc[2] += 1.0;
    if (inf & kWindow) {
      acc[3] += 1.0;
      acc[4] += (r2 > r1) ? 1.0 : 0.0;
      acc[5] += r2;
      acc[6] += r1 + r2;
    }
    if (inf & kPFace) {
      const double P = third * (r1 + r2) + d.G * third * r1 * r2;
      if (x == 0) { acc[7] += P; acc[8] += 1.0; }
      else { acc[9] += P; acc[10] += 1.0; }
    }
    // staggered momentum: both components' momentum with the sign of (-1)^x
    // (resp. y, z), a checkerboard mode the densities do not show
    double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const double t = (double)a[i] + (double)b[i];
      jx += Lat<Q>::ex[i] * t;
      jy += Lat<Q>::ey[i] * t;
      jz += Lat<Q>::ez[i] * t;
    }
    acc[11] += (x & 1) ? -jx : jx;
    acc[12] += (y & 1) ? -jy : jy;
    acc[13] += (z & 1) ? -jz : jz;
  }
  __shared__ double red[4][kObsFields];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kObsFields - 1; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane == 0) red[wave][k] = v;
  }
  for (int o = 32; o > 0; o >>= 1) flags |= __shfl_xor(flags, o, 64);
  if (lane == 0) red[wave][kObsFields - 1] = (double)flags;
  __syncthreads();
  if (threadIdx.x < kObsFields) {
    const int k = threadIdx.x;
    double v;
    if (k == kObsFields - 1) {
      int fl = 0;
      for (int w = 0; w < 4; ++w) fl |= (int)red[w][k];
      v = (double)fl;
    } else {
      v = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
    partials[(int64_t)blockIdx.x * kObsFields + k] = v;
  }
}

// One block of 256 threads per field: thread t sums blocks t, t + 256, ...
// in order, then a fixed tree over the threads -- deterministic.
__global__ void obs_final(const double *__restrict__ partials, int n_blocks, double *__restrict__ out) {
  __shared__ double red[256];
  __shared__ int fred[256];
  const int k = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  int fl = 0;
  for (int b = t; b < n_blocks; b += 256) {
    const double v = partials[(int64_t)b * kObsFields + k];
    if (k == kObsFields - 1) fl |= (int)v;
    else s += v;
  }
  red[t] = s;
  fred[t] = fl;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      red[t] += red[t + o];
      fred[t] |= fred[t + o];
    }
    __syncthreads();
  }
  if (t == 0) out[k] = (k == kObsFields - 1) ? (double)fred[0] : red[0];
}

// ---------------------------------------------------------------------------
// densities as dense float fields
// ---------------------------------------------------------------------------
template <int Q, int ST>
__global__ void density_kernel(const InstDev *__restrict__ insts, int parity, float *__restrict__ dst) {
  const InstDev &d = insts[0];
  gcf *fin = G(d.f[parity]);
  const int64_t n_nodes = (int64_t)d.nx * d.ny * d.nz;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < n_nodes;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int x = n % d.nx;
    const int64_t yz = n / d.nx;
    const int y = yz % d.ny, z = yz / d.ny;
    const uint32_t inf = d.info[x + (int64_t)d.pitch * yz];
    float r1 = 0.f, r2 = 0.f;
    if (!(inf & kSolid)) {
      float a[Q], b[Q];
      if (d.compact) cgather<Q, ST, double>(d, fin, inf, x, y, z, crank(d, x, yz), a, b);
      else gather<Q, ST, double>(d, fin, inf, x, y, z, a, b);
      r1 = (float)sum_q<Q, double>(a);
      r2 = (float)sum_q<Q, double>(b);
    }
    dst[n] = r1;
    dst[n_nodes + n] = r2;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int obs_blocks(const InstDev &h) {
  const int64_t n = (int64_t)h.nx * h.ny * h.nz;
  int64_t b = (n + 255) / 256;
  if (b > 2048) b = 2048;
  return (int)(b < 1 ? 1 : b);
}

static int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_init(const InstDev *d_inst, const InstDev &h, const float *rho0, int parity,
                       hipStream_t s) {
  const int g = grid_for((int64_t)h.nx * h.ny * h.nz);
  if (h.q == 9) {
    if (h.storage == 0) init_kernel<9, 0><<<g, 256, 0, s>>>(d_inst, rho0, parity);
    else init_kernel<9, 1><<<g, 256, 0, s>>>(d_inst, rho0, parity);
  } else {
    if (h.storage == 0) init_kernel<19, 0><<<g, 256, 0, s>>>(d_inst, rho0, parity);
    else init_kernel<19, 1><<<g, 256, 0, s>>>(d_inst, rho0, parity);
  }
  return hipGetLastError();
}

hipError_t launch_init_sat(const InstDev *d_inst, const InstDev &h, const float *sat, float thr, float major,
                           float minor, int parity, hipStream_t s) {
  const int g = grid_for((int64_t)h.nx * h.ny * h.nz);
  if (h.q == 9) {
    if (h.storage == 0) init_kernel<9, 0><<<g, 256, 0, s>>>(d_inst, nullptr, parity, sat, thr, major, minor);
    else init_kernel<9, 1><<<g, 256, 0, s>>>(d_inst, nullptr, parity, sat, thr, major, minor);
  } else {
    if (h.storage == 0) init_kernel<19, 0><<<g, 256, 0, s>>>(d_inst, nullptr, parity, sat, thr, major, minor);
    else init_kernel<19, 1><<<g, 256, 0, s>>>(d_inst, nullptr, parity, sat, thr, major, minor);
  }
  return hipGetLastError();
}

// Frozen reading of Eq. 17 (ivsd_frozen): the virtual solid density at every
// solid node next to fluid, from the state just set up (the rest equilibria
// w_i rho0, whose node sums are the initial densities), held for every step.
template <int Q, int ST>
__global__ void ivsd_freeze_kernel(const InstDev *__restrict__ insts, int parity) {
  const InstDev &d = insts[0];
  const int64_t n_nodes = (int64_t)d.nx * d.ny * d.nz;
  gcf *fin = G(d.f[parity]);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < n_nodes;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int x = n % d.nx;
    const int64_t yz = n / d.nx;
    const int y = yz % d.ny, z = yz / d.ny;
    const int64_t pi = x + (int64_t)d.pitch * yz;
    const uint32_t nb = d.info[pi];
    if (!(nb & kSolid) || !(nb & kLinkMask)) continue;
    const v2f v = ivsd_value<Q>(d, x, y, z, nb, [&](int xn, int yn, int zn) {
      double r1 = 0, r2 = 0;  // the fluid neighbour's own populations
      if (d.compact) {
        const int64_t c = crank(d, xn, yn + (int64_t)d.ny * zn);
        for (int i = 0; i < Q; ++i) {
          r1 += cpop_get<Q, ST>(fin, d.cpitch, 0, i, c);
          r2 += cpop_get<Q, ST>(fin, d.cpitch, 1, i, c);
        }
      } else {
        const int64_t row = yn * d.ystride + zn * d.zstride;
        for (int i = 0; i < Q; ++i) {
          r1 += pop_get<Q, ST>(fin, d.pitch, 0, i, row, xn);
          r2 += pop_get<Q, ST>(fin, d.pitch, 1, i, row, xn);
        }
      }
      return v2f{(float)r1, (float)r2};
    });
    float *out = const_cast<float *>(d.ivsd0);
    out[2 * pi] = v.x;
    out[2 * pi + 1] = v.y;
  }
}

hipError_t launch_ivsd_freeze(const InstDev *d_inst, const InstDev &h, int parity, hipStream_t s) {
  const int g = grid_for((int64_t)h.nx * h.ny * h.nz);
  if (h.q == 9) {
    if (h.storage == 0) ivsd_freeze_kernel<9, 0><<<g, 256, 0, s>>>(d_inst, parity);
    else ivsd_freeze_kernel<9, 1><<<g, 256, 0, s>>>(d_inst, parity);
  } else {
    if (h.storage == 0) ivsd_freeze_kernel<19, 0><<<g, 256, 0, s>>>(d_inst, parity);
    else ivsd_freeze_kernel<19, 1><<<g, 256, 0, s>>>(d_inst, parity);
  }
  return hipGetLastError();
}

// One thread: overwrite one stored value of fluid node (x, y, z) in buffer
// `parity` (population s, i with FP32 storage; the density word of component
// s with BF16-deviation storage).  status: 0 written, 1 a solid node.
template <int Q, int ST>
__global__ void poke_kernel(const InstDev *__restrict__ insts, int parity, int x, int y, int z, int s, int i,
                            float v, int32_t *__restrict__ status) {
  const InstDev &d = insts[0];
  const int64_t row = y + (int64_t)d.ny * z;
  if (d.info[x + (int64_t)d.pitch * row] & kSolid) {
    *status = 1;
    return;
  }
  float *b = d.f[parity];
  if (d.compact) {
    const int64_t c = crank(d, x, row);
    if constexpr (ST == 0) b[(int64_t)s * Q * d.cpitch + cslot<Q>((uint32_t)c, i)] = v;
    else b[2 * c + s] = v;
  } else {
    const int64_t rb = y * d.ystride + z * d.zstride;
    if constexpr (ST == 0) b[rb + (int64_t)(s * Q + i) * d.pitch + x] = v;
    else b[rb + 2 * (int64_t)x + s] = v;
  }
  *status = 0;
}

hipError_t launch_poke(const InstDev *d_inst, const InstDev &h, int parity, int x, int y, int z, int s, int i,
                       float v, int32_t *status, hipStream_t st) {
  if (h.q == 9) {
    if (h.storage == 0) poke_kernel<9, 0><<<1, 1, 0, st>>>(d_inst, parity, x, y, z, s, i, v, status);
    else poke_kernel<9, 1><<<1, 1, 0, st>>>(d_inst, parity, x, y, z, s, i, v, status);
  } else {
    if (h.storage == 0) poke_kernel<19, 0><<<1, 1, 0, st>>>(d_inst, parity, x, y, z, s, i, v, status);
    else poke_kernel<19, 1><<<1, 1, 0, st>>>(d_inst, parity, x, y, z, s, i, v, status);
  }
  return hipGetLastError();
}

hipError_t launch_step_srt(const StepLaunch &L, hipStream_t s);
hipError_t launch_step_mrt(const StepLaunch &L, hipStream_t s);
hipError_t launch_step_trt(const StepLaunch &L, hipStream_t s);

hipError_t launch_step(const StepLaunch &L, hipStream_t s) {
  if (L.collision == 0) return launch_step_srt(L, s);
  if (L.collision == 1) return launch_step_mrt(L, s);
  return launch_step_trt(L, s);
}

const char *step_kernel_name(int q, int collision, int storage, int math, int strategy, int ty) {
  static const char *lat[2] = {"d2q9", "d3q19"};
  static const char *coll[3] = {"SRT", "MRT", "TRT"};
  static const char *st[2] = {"f32", "bf16dev"};
  static const char *mt[2] = {"float", "double"};  // indexed by LBM_MATH_F32, LBM_MATH_F64
  static thread_local char buf[128];
  if (strategy == 2)
    snprintf(buf, sizeof buf, "collide_kernel<%d,%s,%s,%s> (+rho_kernel, psi_kernel)", q, coll[collision],
             st[storage], mt[math]);
  else if (strategy == 3)
    snprintf(buf, sizeof buf, "ccollide_kernel<%d,%s,%s,%s> (+crho_kernel, cpsi_kernel)", q, coll[collision],
             st[storage], mt[math]);
  else if (strategy == 4)
    snprintf(buf, sizeof buf, "step_d2q9_list<%s,%s,%s,%d>", coll[collision], st[storage], mt[math], ty);
  else if (strategy == 5 && q == 19)
    snprintf(buf, sizeof buf, "fwd_step_d3q19<%s,%s,%s> (+fwd_rho_kernel, fwd_ivsd_kernel)", coll[collision],
             st[storage], mt[math]);
  else if (strategy == 5)
    snprintf(buf, sizeof buf, "step_d2q9<%s,%s,%s,%d,compact>", coll[collision], st[storage], mt[math], ty);
  else if (q == 9)
    snprintf(buf, sizeof buf, "step_d2q9<%s,%s,%s,%d>", coll[collision], st[storage], mt[math], ty);
  else
    snprintf(buf, sizeof buf, "step_d3q19<%s,%s,%s>", coll[collision], st[storage], mt[math]);
  return buf;
}

hipError_t launch_fwd_rebuild(const InstDev *d_inst, const InstDev &h, int parity, hipStream_t s) {
  if (h.q != 19 || h.nf == 0) return hipSuccess;
  fwd_rho_kernel<19><<<dim3((unsigned)((h.nf + 255) / 256)), dim3(256), 0, s>>>(d_inst, nullptr, h.nf, parity);
  if (h.nbnd) fwd_ivsd_kernel<19><<<dim3((unsigned)((h.nbnd + 255) / 256)), dim3(256), 0, s>>>(d_inst, parity);
  return hipGetLastError();
}

hipError_t launch_observables(const InstDev *d_inst, const InstDev &h, int parity, double *partials,
                              int n_blocks, double *result, hipStream_t s) {
  if (h.q == 9) {
    if (h.storage == 0) obs_kernel<9, 0><<<n_blocks, 256, 0, s>>>(d_inst, parity, partials);
    else obs_kernel<9, 1><<<n_blocks, 256, 0, s>>>(d_inst, parity, partials);
  } else {
    if (h.storage == 0) obs_kernel<19, 0><<<n_blocks, 256, 0, s>>>(d_inst, parity, partials);
    else obs_kernel<19, 1><<<n_blocks, 256, 0, s>>>(d_inst, parity, partials);
  }
  obs_final<<<kObsFields, 256, 0, s>>>(partials, n_blocks, result);
  return hipGetLastError();
}

hipError_t launch_density(const InstDev *d_inst, const InstDev &h, int parity, float *dst, hipStream_t s) {
  const int g = grid_for((int64_t)h.nx * h.ny * h.nz);
  if (h.q == 9) {
    if (h.storage == 0) density_kernel<9, 0><<<g, 256, 0, s>>>(d_inst, parity, dst);
    else density_kernel<9, 1><<<g, 256, 0, s>>>(d_inst, parity, dst);
  } else {
    if (h.storage == 0) density_kernel<19, 0><<<g, 256, 0, s>>>(d_inst, parity, dst);
    else density_kernel<19, 1><<<g, 256, 0, s>>>(d_inst, parity, dst);
  }
  return hipGetLastError();
}

}  // namespace lbm
