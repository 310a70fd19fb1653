// Step kernels of the two-component LBM for gfx950 (D2Q9 and D3Q19) and
// their launchers, shared by the translation units that instantiate them for
// one collision operator each (lbm_step_srt.hip, lbm_step_mrt.hip,
// lbm_step_trt.hip) and by lbm_kernels.hip (set-up, observables, densities).
#pragma once
// State between steps: the post-collision populations f*^s_i(x), two buffers
// in ping-pong, in a row-interleaved structure of arrays: for each (z, y) row a
// block holding, population after population, one value per x (row pitch a
// multiple of 64).  Accesses stay coalesced along x and the pulls of a wave
// touch a few contiguous row blocks instead of 2Q planes far apart.
// One step pulls f(x) = f*(x - e_i) (bounce-back from solid sources), completes
// the inlet/outlet links, forms the densities, the solid pseudopotential,
// the interaction force and the collision, and writes f* to the other buffer.
// The force at x needs psi within one node, psi at a solid node needs rho
// within one more (Eq. 17), and rho needs the pull: each block therefore
// recomputes densities on a two-node halo around its tile in LDS.
//
// Populations are loaded and stored as float (or BF16 deviations); the node
// arithmetic runs in R = double (default) or float.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lattice.h"
#include "lbm_device.h"

namespace lbm {

template <typename R> struct Vec2 { R x, y; };

// global-memory views of the state (lets the compiler emit global, not flat, accesses)
typedef __attribute__((address_space(1))) float gf;
typedef __attribute__((address_space(1))) const float gcf;
typedef __attribute__((address_space(1))) const uint32_t gcu32;
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) const uint16_t gcu16;

__device__ __forceinline__ gcf *G(const float *p) { return (gcf *)p; }
__device__ __forceinline__ gf *G(float *p) { return (gf *)p; }

// Access at a wave-uniform base plus a per-lane 32-bit byte offset: the
// compiler can then keep the base in scalar registers and address with one
// 32-bit VGPR (global_load ... v_off, s[base]) instead of a 64-bit VGPR pair.
typedef __attribute__((address_space(1))) const char gcc;
typedef __attribute__((address_space(1))) char gc;
__device__ __forceinline__ float ldg(gcf *base, uint32_t boff) { return *(gcf *)((gcc *)base + boff); }
__device__ __forceinline__ void stg(gf *base, uint32_t boff, float v) { *(gf *)((gc *)base + boff) = v; }
// Non-temporal store: for the 3D split steps' post-collision stream, which is
// not read again before the caches have turned over (the next step's density
// kernel starts after the whole GB-sized buffer is written), so keeping it
// in L2 only evicts the pull and psi working sets.  (The 2D steps re-read
// their cache-resident buffers and are slower with it.)
__device__ __forceinline__ void stg_nt(gf *base, uint32_t boff, float v) {
  __builtin_nontemporal_store(v, (gf *)((gc *)base + boff));
}

// ---------------------------------------------------------------------------
// population access by storage kind; a node is addressed by its row block
// offset `row` (y * ystride + z * zstride, in floats) and its x
// FP32:  row block = [s][i][pitch] floats
// BF16:  row block = [pitch] (rho1, rho2) float pairs, then [i-1][pitch]
//        32-bit words holding both components' bf16 deviations
//        d_i = f*_i - w_i rho (i >= 1; component 1 in the low half);
//        f*_0 = rho - sum_i f*_i.  A pull of link i reads one float pair
//        and one word for both components.
// ---------------------------------------------------------------------------
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const v2f gcv2f;
typedef __attribute__((address_space(1))) v2f gv2f;

// The virtual solid density kept for every step under the frozen reading
// of Eq. 17 (ivsd_frozen: evaluated once, on the initial densities), at
// dense index pi.
__device__ __forceinline__ v2f ivsd_held(const InstDev &d, int64_t pi) {
  return ((gcv2f *)d.ivsd0)[pi];
}

template <int Q>
__device__ __forceinline__ float bf16_pop(gcf *__restrict__ b, int pitch, int s, int i, int64_t row, int x,
                                          float r) {
  gcu16 *dv = (gcu16 *)b;
  const int64_t k = 2 * (row + (int64_t)(1 + i) * pitch + x) + s;
  return __builtin_fmaf((float)Lat<Q>::w[i], r, bf16_to_f32(dv[k]));
}

template <int Q, int ST>
__device__ __forceinline__ float pop_get(gcf *__restrict__ b, int pitch, int s, int i, int64_t row, int x) {
  if constexpr (ST == 0) {
    return b[row + (int64_t)(s * Q + i) * pitch + x];
  } else {
    const float r = b[row + 2 * (int64_t)x + s];
    if (i == 0) {
      // the rest population closes the node's mass: rho - sum of the others,
      // reconstructed exactly as a pull elsewhere reconstructs them
      float sum = 0.f;
#pragma unroll
      for (int j = 1; j < Q; ++j) sum += bf16_pop<Q>(b, pitch, s, j, row, x, r);
      return r - sum;
    }
    return bf16_pop<Q>(b, pitch, s, i, row, x, r);
  }
}

// Both components' link i of one node (the same values as two pop_get
// calls, from one float-pair and one word load per link in BF16).
template <int Q, int ST>
__device__ __forceinline__ void pop_get2(gcf *__restrict__ b, int pitch, int i, int64_t row, int x, float &f0,
                                         float &f1) {
  if constexpr (ST == 0) {
    f0 = pop_get<Q, 0>(b, pitch, 0, i, row, x);
    f1 = pop_get<Q, 0>(b, pitch, 1, i, row, x);
  } else {
    const v2f r = *(gcv2f *)(b + row + 2 * (int64_t)x);
    auto link = [&](int j, float &g0, float &g1) {
      const uint32_t u = *(gcu32 *)(b + row + (int64_t)(1 + j) * pitch + x);
      const float w = (float)Lat<Q>::w[j];
      g0 = __builtin_fmaf(w, r.x, bf16_to_f32((uint16_t)(u & 0xffffu)));
      g1 = __builtin_fmaf(w, r.y, bf16_to_f32((uint16_t)(u >> 16)));
    };
    if (i == 0) {
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int j = 1; j < Q; ++j) {
        float g0, g1;
        link(j, g0, g1);
        s0 += g0;
        s1 += g1;
      }
      f0 = r.x - s0;
      f1 = r.y - s1;
    } else {
      link(i, f0, f1);
    }
  }
}

// Store both components' post-collision populations of one node (NT:
// non-temporal FP32 stores).
template <int Q, int ST, bool NT = false>
__device__ __forceinline__ void pop_store(gf *__restrict__ b, int pitch, int64_t row, int x,
                                          const float (&f0)[Q], const float (&f1)[Q], float rho1,
                                          float rho2) {
  if constexpr (ST == 0) {
    const uint32_t bo = (uint32_t)x * 4u;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if constexpr (NT) {
        stg_nt(b + row + (int64_t)i * pitch, bo, f0[i]);
        stg_nt(b + row + (int64_t)(Q + i) * pitch, bo, f1[i]);
      } else {
        stg(b + row + (int64_t)i * pitch, bo, f0[i]);
        stg(b + row + (int64_t)(Q + i) * pitch, bo, f1[i]);
      }
    }
  } else {
    // collision conserves each component's node mass, so rho is stored as is
    *(gv2f *)(b + row + 2 * (int64_t)x) = v2f{rho1, rho2};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const float w = (float)Lat<Q>::w[i];
      const uint32_t u = (uint32_t)f32_to_bf16(f0[i] - w * rho1) | ((uint32_t)f32_to_bf16(f1[i] - w * rho2) << 16);
      *(gu32 *)(b + row + (int64_t)(1 + i) * pitch + x) = u;
    }
  }
}

// Inlet/outlet completion of one pulled node (links already pulled).
template <int Q, int ST, typename R>
__device__ __forceinline__ void complete(const InstDev &d, gcf *__restrict__ fin, uint32_t info, int x,
                                         int y, int z, float (&f0)[Q], float (&f1)[Q]) {
  const int t = y + d.ny * z;
  const int64_t nt = (int64_t)d.ny * d.nz;
  const int64_t row = y * d.ystride + z * d.zstride;
  gcf *frz = G(d.frozen);
  complete_boundary<Q, R>(
      d, info, f0, f1, [&](int s, int i) { return pop_get<Q, ST>(fin, d.pitch, s, i, row, x); },
      [&](int s, int i) { return frz[(int64_t)(s * Q + i) * nt + t]; });
}

// ---------------------------------------------------------------------------
// Streaming.  f_i(x) = f*_i(x - e_i), or f*_opp(i)(x) where x - e_i is solid.
// FP32 storage keeps the bounce-back values in ghost slots: when fluid node x
// stores its post-collision state, it also writes f*_opp(i)(x) into link i's
// slot of each solid source node x - e_i.  A slot (i, s) of a solid node s has
// exactly one writer (x = s + e_i), so every pull is the uniform
// f_i(x) = buf[i][x - e_i].  BF16 storage reads the node's own opposite slot.
// Sources wrap periodically; a wrapped source across an open face is a
// missing link whose value the inlet/outlet completion overwrites.
// ---------------------------------------------------------------------------

// Source row offsets (in floats) for a node row (y, z): src[ey+1][ez+1] is
// the row of (y - ey, z - ez) with periodic wrap.  Uniform across a wave when
// y and z are.
// A value the caller knows to be equal across the wave, marked as such so
// that addresses built from it stay in scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// UNI: the caller guarantees (y, z) is the same for every active lane.
template <int Q, bool UNI = false>
__device__ __forceinline__ void source_rows(const InstDev &d, int y, int z, int64_t (&src)[3][3]) {
  const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? d.nz - 1 : z - 1, zp = z == d.nz - 1 ? 0 : z + 1;
  const int ys[3] = {yp, y, ym}, zs[3] = {zp, z, zm};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int64_t v = ys[a] * d.ystride + zs[b] * d.zstride;
      src[a][b] = UNI ? uniform64(v) : v;
    }
}

// Source x for e_x = -1, 0, +1 (periodic wrap).
__device__ __forceinline__ void source_x(const InstDev &d, int x, int (&xs)[3]) {
  xs[0] = x == d.nx - 1 ? 0 : x + 1;
  xs[1] = x;
  xs[2] = x == 0 ? d.nx - 1 : x - 1;
}

// Pull both components at (x, row src[1][1]) given its source rows.
template <int Q, int ST>
__device__ __forceinline__ void pull_row(const InstDev &d, gcf *__restrict__ fin, uint32_t info,
                                         const int64_t (&src)[3][3], const int (&xs)[3], float (&f0)[Q],
                                         float (&f1)[Q]) {
  using L = Lat<Q>;
  const int pitch = __builtin_amdgcn_readfirstlane(d.pitch);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int64_t row = src[L::ey[i] + 1][L::ez[i] + 1];
    const int sx = xs[L::ex[i] + 1];
    if constexpr (ST == 0) {
      gcf *b = fin + row + (int64_t)i * pitch;
      const uint32_t bo = (uint32_t)sx * 4u;
      f0[i] = ldg(b, bo);
      f1[i] = ldg(b + (int64_t)Q * pitch, bo);
    } else {
      const bool bb = (info >> i) & 1u;
      const int64_t r = bb ? src[1][1] : row;
      const int x = bb ? xs[1] : sx;
      const int pi = bb ? L::opp[i] : i;
      pop_get2<Q, 1>(fin, pitch, pi, r, x, f0[i], f1[i]);
    }
  }
}

// Ghost slots (FP32 storage): link i of each solid source x - e_i receives f*_opp(i)(x).
template <int Q, int ST>
__device__ __forceinline__ void store_ghosts(const InstDev &d, gf *__restrict__ fout, uint32_t info,
                                             const int64_t (&src)[3][3], const int (&xs)[3],
                                             const float (&f0)[Q], const float (&f1)[Q]) {
  if constexpr (ST == 0) {
    using L = Lat<Q>;
    if (!(info & kLinkMask)) return;
    const int pitch = d.pitch;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if (info & (1u << i)) {
        gf *b = fout + src[L::ey[i] + 1][L::ez[i] + 1] + (int64_t)i * pitch;
        const uint32_t bo = (uint32_t)xs[L::ex[i] + 1] * 4u;
        stg(b, bo, f0[L::opp[i]]);
        stg(b + (int64_t)Q * pitch, bo, f1[L::opp[i]]);
      }
    }
  }
}

// Pull + completion for one fluid node at in-domain (x, y, z) (per-lane rows).
template <int Q, int ST, typename R>
__device__ __forceinline__ void gather(const InstDev &d, gcf *__restrict__ fin, uint32_t info,
                                       int x, int y, int z, float (&f0)[Q], float (&f1)[Q]) {
  int64_t src[3][3];
  int xs[3];
  source_rows<Q>(d, y, z, src);
  source_x(d, x, xs);
  pull_row<Q, ST>(d, fin, info, src, xs, f0, f1);
  if (info & (kInlet | kOutlet)) complete<Q, ST, R>(d, fin, info, x, y, z, f0, f1);
}

// Periodic image of a tile-region coordinate.  A tile's halo (and the
// unused tail of the last tile) can lie more than one period away when the
// periodic extent is smaller than the tile, so this is a true modulo.
__device__ __forceinline__ int wrap_index(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Blocks are dealt round-robin to the 8 XCDs; renumber them so each XCD
// works on a contiguous range of tiles and neighbouring tiles share its L2.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
  return xcd * q8 + min(xcd, r8) + (b >> 3);
}

// The same, walking the tiles in reverse on odd steps: a step's first tiles
// are then the ones the previous step wrote last, which are still in the
// Infinity Cache when a batch's buffers exceed it (64 uneven D2Q9 instances:
// 0.483 -> 0.466 ms per step).
__device__ __forceinline__ int xcd_block_alternating(int parity) {
  const int b = xcd_block();
  return (parity & 1) ? (int)gridDim.x - 1 - b : b;
}

// The compacted layout's tables are read through global-address loads: a
// flat load would also count against the scalar-load counter, so that every
// wait for an instance field (scalar loads) would wait for it as well.
// Only the low word of a row word's prefix is loaded (compact indices stay
// below 2^32): a 16-byte load whose last register the code never reads would
// make the compiler wait for the load before reusing that register.
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef __attribute__((address_space(1))) const u32x3 gcu32x3;
__device__ __forceinline__ RowWord row_word(const InstDev &d, int64_t i) {
  const u32x3 v = *(gcu32x3 *)((gcu32 *)d.cword + 4 * i);
  return RowWord{(unsigned long long)v.x | ((unsigned long long)v.y << 32), (long long)v.z};
}
__device__ __forceinline__ uint32_t gld32(const uint32_t *p, int64_t i) { return ((gcu32 *)p)[i]; }

// Compact index of fluid node (x, row), row = y + ny * z.  For a solid
// position it is the index of the next fluid node (at most nf).
__device__ __forceinline__ int64_t crank(const InstDev &d, int x, int64_t row) {
  const RowWord w = row_word(d, row * (d.pitch >> 6) + (x >> 6));
  const unsigned long long below = (1ull << (x & 63)) - 1ull;
  return w.pre + __popcll(w.bits & below);
}

// FP32 populations of the compacted layout: per component, blocks of 64
// consecutive fluid nodes, each holding its Q link rows, f*[s][c / 64][i][c %
// 64] (component s starts Q * cpitch floats in).  The 64 nodes of a wave
// find all their links in one 64 x Q x 4-byte block per component instead
// of Q planes spread over the buffer (measured for D3Q19 at 384^3: the
// compacted split step 3.7 % faster than with whole-buffer link planes).
// cslot is the float offset within a component; byte offsets stay below
// Q * cpitch * 4 < 2^32, as the host requires.  BF16 storage keeps link
// planes over the whole buffer.
template <int Q>
__device__ __forceinline__ uint32_t cslot(uint32_t c, int i) {
  return (c & ~63u) * (uint32_t)Q + (uint32_t)i * 64u + (c & 63u);
}
template <int Q, int ST>
__device__ __forceinline__ float cpop_get(gcf *__restrict__ b, int cp, int s, int i, int64_t c) {
  if constexpr (ST == 0) return b[(int64_t)s * Q * cp + cslot<Q>((uint32_t)c, i)];
  else return pop_get<Q, ST>(b, cp, s, i, 0, (int)c);
}
template <int Q, int ST, bool NT = false>
__device__ __forceinline__ void cpop_store(gf *__restrict__ b, int cp, int64_t c, const float (&f0)[Q],
                                           const float (&f1)[Q], float rho1, float rho2) {
  if constexpr (ST == 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const uint32_t bo = cslot<Q>((uint32_t)c, i) * 4u;
      if constexpr (NT) {
        stg_nt(b, bo, f0[i]);
        stg_nt(b + (int64_t)Q * cp, bo, f1[i]);
      } else {
        stg(b, bo, f0[i]);
        stg(b + (int64_t)Q * cp, bo, f1[i]);
      }
    }
  } else {
    pop_store<Q, ST>(b, cp, 0, (int)c, f0, f1, rho1, rho2);
  }
}

// Pull of D2Q9 fluid node (x, y) in the compacted layout (populations of the
// fluid nodes only, see cslot); c receives the node's compact index.
// The rank of column x in each source row gives every fluid source's index
// (x - 1: rank - 1; x + 1: rank + the column's fluid bit); bounce-back reads
// the node's own opposite slot; wrapped x sources are ranked directly.
template <int ST>
__device__ __forceinline__ void cpull9(const InstDev &d, gcf *__restrict__ fin, uint32_t info, int x, int y,
                                       const int (&xs)[3], int32_t &c, float (&f0)[9], float (&f1)[9]) {
  using L = Lat<9>;
  const int cp = d.cpitch, ny = d.ny;
  const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};  // y - e_y, by e_y + 1
  const int64_t wpr = d.pitch >> 6;
  const unsigned long long below = (1ull << (x & 63)) - 1ull;
  int32_t rk[3];
  int fl[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const RowWord w = row_word(d, ys[a] * wpr + (x >> 6));
    rk[a] = (int32_t)(w.pre + __popcll(w.bits & below));
    fl[a] = (int)((w.bits >> (x & 63)) & 1ull);
  }
  c = rk[1];
  const bool x_edge = x == 0 || x == d.nx - 1;
  const int32_t last = (int32_t)(d.nf - 1);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int32_t sc = c;
    int pi = i;
    if (i != 0) {
      if ((info >> i) & 1u) {
        pi = L::opp[i];
      } else {
        const int a = L::ey[i] + 1;
        if (L::ex[i] == 0) {
          sc = rk[a];
        } else if (!x_edge) {
          sc = L::ex[i] > 0 ? rk[a] - 1 : rk[a] + fl[a];
        } else {
          // wrapped source: periodic x, or a missing link at an open face
          // (an arbitrary node, overwritten by the completion below)
          const int32_t r = (int32_t)crank(d, xs[L::ex[i] + 1], ys[a]);
          sc = r < last ? r : last;
        }
      }
    }
    if constexpr (ST == 0) {
      const uint32_t bo = cslot<9>((uint32_t)sc, pi) * 4u;
      f0[i] = ldg(fin, bo);
      f1[i] = ldg(fin + (int64_t)9 * cp, bo);
    } else {
      pop_get2<9, ST>(fin, cp, pi, 0, (int)sc, f0[i], f1[i]);
    }
  }
}

// Inlet/outlet completion of a D2Q9 node pulled by cpull9 (compact index c).
template <int ST, typename R>
__device__ __forceinline__ void ccomplete9(const InstDev &d, gcf *__restrict__ fin, uint32_t info, int y,
                                           int32_t c, float (&f0)[9], float (&f1)[9]) {
  gcf *frz = G(d.frozen);
  const int cp = d.cpitch, ny = d.ny;
  complete_boundary<9, R>(
      d, info, f0, f1, [&](int s, int i) { return cpop_get<9, ST>(fin, cp, s, i, c); },
      [&](int s, int i) { return frz[(int64_t)(s * 9 + i) * ny + y]; });
}

// ---------------------------------------------------------------------------
// D2Q9 fused step.  Block = 4 waves over a region of 64 columns x (TY + 4)
// rows: 60 x TY interior nodes plus a 2-node halo.  Wave w owns interior rows
// 2 + w + 4k (k < TY/4) and one halo row; a row is wave-uniform, so every pull
// is one load from a scalar row base plus the lane's x.
// Phase 1: pull + complete + densities for all region nodes -> LDS.
// Phase 2: virtual solid density (Eq. 17) in place at solid region nodes.
// Phase 3: force (Eq. 13 with the open-face mirror) and collision for the
//          interior nodes, whose pulled populations stayed in registers.
// ---------------------------------------------------------------------------
// Occupancy: the step is bound by the latency of its memory chain, so
// resident waves count (the 64-instance batch at TY = 12 takes 15 % longer
// with three blocks per CU than with four, 49 % with two).  TY = 12 parks
// the last interior row of each wave in LDS between the phases, which fits
// it in 128 registers and 26 KB of LDS (four waves per SIMD).  With FP32
// node arithmetic and FP32 storage TY = 8 parks its last row as well and
// fits 80 registers: six waves per SIMD (measured 5 % faster on the batch
// and 7 % on a 1024 x 512 instance than four waves with every row in
// registers); otherwise it keeps every pulled row in registers at four waves.
template <int TY, typename R, int ST> struct FusedShape {
  static constexpr bool kF32 = sizeof(R) == 4 && ST == 0;
  static constexpr int kParked = (TY == 12 || (TY == 8 && kF32)) ? 1 : 0;  // interior rows per wave kept in LDS
  static constexpr int kWaves = TY == 16 ? 1 : ((TY == 8 && kF32) ? 6 : 4);
};

// CL = 1: the same step over the compacted layout (fluid nodes only stored,
// pulls by rank, bounce-back from the node's own slots, no ghost slots).
template <int COLL, int ST, typename R, int TY, int CL = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FusedShape<TY, R, ST>::kWaves))) void step_d2q9(
    const InstDev *__restrict__ insts, const int32_t *__restrict__ block_inst, int parity) {
  using L = Lat<9>;
  using V = Vec2<R>;
  constexpr int KR = TY / 4;        // interior rows per wave
  constexpr int kRH = TY + 4;       // region rows
  constexpr int KP = FusedShape<TY, R, ST>::kParked;
  __shared__ V psi[kRH][64];
  __shared__ float park[KP > 0 ? KP * 4 : 1][18][64];  // [row slot * 4 + wave][component * 9 + link][lane]

  const int bid = xcd_block_alternating(parity);
  const int inst = __builtin_amdgcn_readfirstlane(block_inst ? block_inst[bid] : 0);
  const InstDev &d = insts[inst];
  const int lb = bid - d.block_base;
  const int tx = lb % d.tiles_x, ty = lb / d.tiles_x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  gcf *__restrict__ fin = G(d.f[parity]);
  gf *__restrict__ fout = G(d.f[parity ^ 1]);
  gcu32 *__restrict__ infop = (gcu32 *)d.info;
  const int nx = d.nx, ny = d.ny;
  const bool px = d.periodic & 1, py = d.periodic & 2;

  // region column of this lane
  int gx = tx * kTileX - 2 + lane;
  const bool col_store = lane >= 2 && lane < 62 && gx < nx;
  bool col_in = true;
  if (gx < 0 || gx >= nx) {
    if (px) gx = wrap_index(gx, nx);
    else col_in = false;
  }
  const int gxa = col_in ? gx : (gx < 0 ? 0 : nx - 1);
  int xs[3];
  source_x(d, gxa, xs);

  // rows owned (wave-uniform): k < KR interior (2 + wave + 4k), k = KR halo
  int rows[KR + 1], gy[KR + 1];
  bool row_in[KR + 1];
#pragma unroll
  for (int k = 0; k <= KR; ++k) {
    rows[k] = k < KR ? 2 + wave + 4 * k : (wave < 2 ? wave : TY + wave);
    int y = ty * TY - 2 + rows[k];
    bool in = true;
    if (y < 0 || y >= ny) {
      if (py) y = wrap_index(y, ny);
      else in = false;
    }
    gy[k] = in ? y : 0;
    row_in[k] = in;
  }
  uint32_t info[KR + 1];
#pragma unroll
  for (int k = 0; k <= KR; ++k)
    info[k] = (row_in[k] && col_in) ? infop[gx + (int64_t)d.pitch * gy[k]] : kSolid;

  // Phase 1: issue every pull of this thread, then complete and sum.  Solid
  // and out-of-domain lanes read valid addresses in the same rows and discard
  // them (the BF16 layout pulls only for fluid lanes, to bound the loads in
  // flight).
  float f0[KR][9], f1[KR][9], h0[9], h1[9];
  int64_t srow[KR + 1][3][3];
  int32_t cidx[KR + 1];  // compact indices (CL)
  if constexpr (CL) {
#pragma unroll
    for (int k = 0; k <= KR; ++k) {
      float(&a)[9] = k < KR ? f0[k < KR ? k : 0] : h0;
      float(&b)[9] = k < KR ? f1[k < KR ? k : 0] : h1;
      cidx[k] = 0;
      if (!(info[k] & kSolid)) cpull9<ST>(d, fin, info[k], gx, gy[k], xs, cidx[k], a, b);
    }
  } else {
#pragma unroll
    for (int k = 0; k <= KR; ++k) source_rows<9, true>(d, gy[k], 0, srow[k]);
#pragma unroll
    for (int k = 0; k < KR; ++k)
      if (ST == 0 || !(info[k] & kSolid)) pull_row<9, ST>(d, fin, info[k], srow[k], xs, f0[k], f1[k]);
    if (ST == 0 || !(info[KR] & kSolid)) pull_row<9, ST>(d, fin, info[KR], srow[KR], xs, h0, h1);
  }
#pragma unroll
  for (int k = 0; k <= KR; ++k) {
    R rho1 = 0, rho2 = 0;
    if (!(info[k] & kSolid)) {
      float(&a)[9] = k < KR ? f0[k < KR ? k : 0] : h0;
      float(&b)[9] = k < KR ? f1[k < KR ? k : 0] : h1;
      if (info[k] & (kInlet | kOutlet)) {
        if constexpr (CL) ccomplete9<ST, R>(d, fin, info[k], gy[k], cidx[k], a, b);
        else complete<9, ST, R>(d, fin, info[k], gx, gy[k], 0, a, b);
      }
      rho1 = sum_q<9, R>(a);
      rho2 = sum_q<9, R>(b);
    } else if (d.ivsd0 && row_in[k] && col_in && (info[k] & kLinkMask)) {
      // frozen reading of Eq. 17: the held value (phase 2 then skips)
      const v2f h = ivsd_held(d, (uint32_t)gx + (uint32_t)d.pitch * (uint32_t)gy[k]);
      rho1 = (R)h.x;
      rho2 = (R)h.y;
    }
    psi[rows[k]][lane] = V{rho1, rho2};
    if (k >= KR - KP && k < KR) {
      float(&pk)[18][64] = park[(k - (KR - KP)) * 4 + wave];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        pk[i][lane] = f0[k < KR ? k : 0][i];
        pk[9 + i][lane] = f1[k < KR ? k : 0][i];
      }
    }
  }
  __syncthreads();

  // Phase 2: psi at solid nodes = chi^s * weighted mean of fluid-neighbour rho^s
  // (under the frozen reading of Eq. 17 phase 1 has put the held values)
  const bool held = d.ivsd0 != nullptr;
#pragma unroll
  for (int k = 0; k <= KR; ++k) {
    const int r = rows[k];
    if (held || !row_in[k] || !col_in || !(info[k] & kSolid) || r < 1 || r > kRH - 2 || lane < 1 || lane > 62)
      continue;
    const uint32_t nb = info[k];
    if (!(nb & kLinkMask)) continue;
    R s1 = 0, s2 = 0, den = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      if (nb & (1u << i)) {
        const V p = psi[r + L::ey[i]][lane + L::ex[i]];
        const R w = (R)L::w[i];
        s1 += w * p.x;
        s2 += w * p.y;
        den += w;
      }
    }
    const R inv = rcp<R>(den);
    psi[r][lane] = V{(R)d.chi1 * s1 * inv, (R)d.chi2 * s2 * inv};
  }
  __syncthreads();

  // Phase 3: force + collision for interior rows
  const R w1 = R(1.0 / 9.0), w5 = R(1.0 / 36.0);
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int r = rows[k];
    const int gy_raw = ty * TY - 2 + r;
    if (!row_in[k] || !col_store || gy_raw >= ny || (info[k] & kSolid)) continue;
    const uint32_t inf = info[k];
    const V c = psi[r][lane];
    const R rho1 = c.x, rho2 = c.y;
    // sum_i w_i psi(x + e_i) e_i by opposite pairs
    R sx1, sy1, sx2, sy2;  // sums of component 1's / 2's psi
    {
      const V p2 = psi[r + 1][lane], p4 = psi[r - 1][lane];
      if (inf & (kInlet | kOutlet)) {
        // mirrored neighbours cancel every pair with an x component
        sx1 = 0;
        sx2 = 0;
        sy1 = w1 * (p2.x - p4.x);
        sy2 = w1 * (p2.y - p4.y);
      } else {
        const V p1 = psi[r][lane + 1], p3 = psi[r][lane - 1];
        const V p5 = psi[r + 1][lane + 1], p7 = psi[r - 1][lane - 1];
        const V p6 = psi[r + 1][lane - 1], p8 = psi[r - 1][lane + 1];
        const R a57 = p5.x - p7.x, a68 = p6.x - p8.x;
        const R b57 = p5.y - p7.y, b68 = p6.y - p8.y;
        sx1 = w1 * (p1.x - p3.x) + w5 * (a57 - a68);
        sy1 = w1 * (p2.x - p4.x) + w5 * (a57 + a68);
        sx2 = w1 * (p1.y - p3.y) + w5 * (b57 - b68);
        sy2 = w1 * (p2.y - p4.y) + w5 * (b57 + b68);
      }
    }
    const R G_ = (R)d.G, gxb = (R)d.gx, gyb = (R)d.gy;
    const R F1x = -G_ * rho1 * sx2 + rho1 * gxb, F1y = -G_ * rho1 * sy2 + rho1 * gyb;
    const R F2x = -G_ * rho2 * sx1 + rho2 * gxb, F2y = -G_ * rho2 * sy1 + rho2 * gyb;
    if (k >= KR - KP) {
      const float(&pk)[18][64] = park[(k - (KR - KP)) * 4 + wave];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        f0[k][i] = pk[i][lane];
        f1[k][i] = pk[9 + i][lane];
      }
    }
    collide_node<9, COLL, R>(d, f0[k], f1[k], rho1, rho2, F1x, F1y, R(0), F2x, F2y, R(0));
    if constexpr (CL) {
      cpop_store<9, ST>(fout, d.cpitch, cidx[k], f0[k], f1[k], (float)rho1, (float)rho2);
    } else {
      pop_store<9, ST>(fout, d.pitch, uniform64(gy_raw * d.ystride), gx, f0[k], f1[k], (float)rho1, (float)rho2);
      store_ghosts<9, ST>(d, fout, inf, srow[k], xs, f0[k], f1[k]);
    }
  }
}

// ---------------------------------------------------------------------------
// D2Q9 fused step with a listed collision phase.  Phases 1 and 2 as in the
// fused step; in phase 1 every interior fluid node also parks its pulled
// (and completed) populations and its info word in LDS, dense by interior
// position.  Phase 3 runs over a per-tile list of the fluid interior nodes
// (row-major, built from ballots and a fixed-order prefix in LDS), one list
// entry per thread, so no lane spends the collision on a solid node.  The
// arithmetic is the fused step's, value for value.
// LDS: populations 72 B per interior node (34.6 KB at TY = 8) + densities.
// ---------------------------------------------------------------------------
template <int COLL, int ST, typename R, int TY>
__global__ __launch_bounds__(256) void step_d2q9_list(const InstDev *__restrict__ insts,
                                                      const int32_t *__restrict__ block_inst, int parity) {
  using L = Lat<9>;
  using V = Vec2<R>;
  constexpr int KR = TY / 4;
  constexpr int kRH = TY + 4;
  constexpr int kN = TY * kTileX;   // interior nodes of a tile
  __shared__ V psi[kRH][64];
  __shared__ float pops[18][kN];    // [component * 9 + link][interior position]
  __shared__ uint32_t pinfo[kN];
  __shared__ uint16_t list[kN];     // interior positions of the fluid nodes, row-major
  __shared__ int cnt[TY];

  const int bid = xcd_block_alternating(parity);
  const int inst = __builtin_amdgcn_readfirstlane(block_inst ? block_inst[bid] : 0);
  const InstDev &d = insts[inst];
  const int lb = bid - d.block_base;
  const int tx = lb % d.tiles_x, ty = lb / d.tiles_x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  gcf *__restrict__ fin = G(d.f[parity]);
  gf *__restrict__ fout = G(d.f[parity ^ 1]);
  gcu32 *__restrict__ infop = (gcu32 *)d.info;
  const int nx = d.nx, ny = d.ny;
  const bool px = d.periodic & 1, py = d.periodic & 2;

  int gx = tx * kTileX - 2 + lane;
  const bool col_store = lane >= 2 && lane < 62 && gx < nx;
  bool col_in = true;
  if (gx < 0 || gx >= nx) {
    if (px) gx = wrap_index(gx, nx);
    else col_in = false;
  }
  const int gxa = col_in ? gx : (gx < 0 ? 0 : nx - 1);
  int xs[3];
  source_x(d, gxa, xs);

  int rows[KR + 1], gy[KR + 1];
  bool row_in[KR + 1];
#pragma unroll
  for (int k = 0; k <= KR; ++k) {
    rows[k] = k < KR ? 2 + wave + 4 * k : (wave < 2 ? wave : TY + wave);
    int y = ty * TY - 2 + rows[k];
    bool in = true;
    if (y < 0 || y >= ny) {
      if (py) y = wrap_index(y, ny);
      else in = false;
    }
    gy[k] = in ? y : 0;
    row_in[k] = in;
  }
  uint32_t info[KR + 1];
#pragma unroll
  for (int k = 0; k <= KR; ++k)
    info[k] = (row_in[k] && col_in) ? infop[gx + (int64_t)d.pitch * gy[k]] : kSolid;

  // Phase 1: pull every row of this thread, then complete, sum, and park the
  // interior fluid nodes' populations
  {
    float f0[KR + 1][9], f1[KR + 1][9];
    int64_t srow[KR + 1][3][3];
#pragma unroll
    for (int k = 0; k <= KR; ++k) source_rows<9, true>(d, gy[k], 0, srow[k]);
#pragma unroll
    for (int k = 0; k <= KR; ++k)
      if (ST == 0 || !(info[k] & kSolid)) pull_row<9, ST>(d, fin, info[k], srow[k], xs, f0[k], f1[k]);
#pragma unroll
    for (int k = 0; k <= KR; ++k) {
      R rho1 = 0, rho2 = 0;
      if (!(info[k] & kSolid)) {
        if (info[k] & (kInlet | kOutlet)) complete<9, ST, R>(d, fin, info[k], gx, gy[k], 0, f0[k], f1[k]);
        rho1 = sum_q<9, R>(f0[k]);
        rho2 = sum_q<9, R>(f1[k]);
      }
      psi[rows[k]][lane] = V{rho1, rho2};
      if (k < KR) {
        const bool fluid = row_in[k] && col_store && ty * TY - 2 + rows[k] < ny && !(info[k] & kSolid);
        if (fluid) {
          const int pos = (rows[k] - 2) * kTileX + lane - 2;
#pragma unroll
          for (int i = 0; i < 9; ++i) {
            pops[i][pos] = f0[k][i];
            pops[9 + i][pos] = f1[k][i];
          }
          pinfo[pos] = info[k];
        }
        const unsigned long long m = __ballot(fluid);
        if (lane == 0) cnt[rows[k] - 2] = __popcll(m);
      }
    }
  }
  __syncthreads();

  // Phase 2: virtual solid density; the list of fluid interior nodes
#pragma unroll
  for (int k = 0; k <= KR; ++k) {
    const int r = rows[k];
    const uint32_t nb = info[k];
    if (k < KR) {
      const bool fluid = row_in[k] && col_store && ty * TY - 2 + r < ny && !(nb & kSolid);
      const unsigned long long m = __ballot(fluid);
      int base = 0;
      for (int q = 0; q < r - 2; ++q) base += cnt[q];
      if (fluid) list[base + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)((r - 2) * kTileX + lane - 2);
    }
    if (!row_in[k] || !col_in || !(nb & kSolid) || r < 1 || r > kRH - 2 || lane < 1 || lane > 62) continue;
    if (!(nb & kLinkMask)) continue;
    if (d.ivsd0) {  // frozen reading of Eq. 17: the held value
      const v2f h = ivsd_held(d, gx + (int64_t)d.pitch * gy[k]);
      psi[r][lane] = V{(R)h.x, (R)h.y};
      continue;
    }
    R s1 = 0, s2 = 0, den = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      if (nb & (1u << i)) {
        const V p = psi[r + L::ey[i]][lane + L::ex[i]];
        const R w = (R)L::w[i];
        s1 += w * p.x;
        s2 += w * p.y;
        den += w;
      }
    }
    const R inv = rcp<R>(den);
    psi[r][lane] = V{(R)d.chi1 * s1 * inv, (R)d.chi2 * s2 * inv};
  }
  int total = 0;
#pragma unroll
  for (int q = 0; q < TY; ++q) total += cnt[q];
  __syncthreads();

  // Phase 3: force + collision over the list.  Stores address the tile's
  // first interior row (wave-uniform) plus a 32-bit byte offset; the host
  // keeps TY row blocks within 2^31 bytes for this strategy.
  const R w1 = R(1.0 / 9.0), w5 = R(1.0 / 36.0);
  gf *const tile_out = fout + uniform64((int64_t)ty * TY * d.ystride);
  const int pitch = __builtin_amdgcn_readfirstlane(d.pitch);
  const uint32_t ystride = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)d.ystride);
  for (int t = threadIdx.x; t < total; t += 256) {
    const int pos = list[t];
    const int ri = pos / kTileX, ci = pos - ri * kTileX;
    const int r = ri + 2, ln = ci + 2;
    const int x = tx * kTileX + ci, y = ty * TY + ri;
    const uint32_t inf = pinfo[pos];
    float f0[9], f1[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      f0[i] = pops[i][pos];
      f1[i] = pops[9 + i][pos];
    }
    const V c = psi[r][ln];
    const R rho1 = c.x, rho2 = c.y;
    R sx1, sy1, sx2, sy2;
    {
      const V p2 = psi[r + 1][ln], p4 = psi[r - 1][ln];
      if (inf & (kInlet | kOutlet)) {
        sx1 = 0;
        sx2 = 0;
        sy1 = w1 * (p2.x - p4.x);
        sy2 = w1 * (p2.y - p4.y);
      } else {
        const V p1 = psi[r][ln + 1], p3 = psi[r][ln - 1];
        const V p5 = psi[r + 1][ln + 1], p7 = psi[r - 1][ln - 1];
        const V p6 = psi[r + 1][ln - 1], p8 = psi[r - 1][ln + 1];
        const R a57 = p5.x - p7.x, a68 = p6.x - p8.x;
        const R b57 = p5.y - p7.y, b68 = p6.y - p8.y;
        sx1 = w1 * (p1.x - p3.x) + w5 * (a57 - a68);
        sy1 = w1 * (p2.x - p4.x) + w5 * (a57 + a68);
        sx2 = w1 * (p1.y - p3.y) + w5 * (b57 - b68);
        sy2 = w1 * (p2.y - p4.y) + w5 * (b57 + b68);
      }
    }
    const R G_ = (R)d.G, gxb = (R)d.gx, gyb = (R)d.gy;
    const R F1x = -G_ * rho1 * sx2 + rho1 * gxb, F1y = -G_ * rho1 * sy2 + rho1 * gyb;
    const R F2x = -G_ * rho2 * sx1 + rho2 * gxb, F2y = -G_ * rho2 * sy1 + rho2 * gyb;
    collide_node<9, COLL, R>(d, f0, f1, rho1, rho2, F1x, F1y, R(0), F2x, F2y, R(0));
    if constexpr (ST == 0) {
      const uint32_t bo = ((uint32_t)ri * ystride + (uint32_t)x) * 4u;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        stg(tile_out + (int64_t)i * pitch, bo, f0[i]);
        stg(tile_out + (int64_t)(9 + i) * pitch, bo, f1[i]);
      }
    } else {
      pop_store<9, ST>(fout, d.pitch, y * d.ystride, x, f0, f1, (float)rho1, (float)rho2);
    }
    if (inf & kLinkMask) {
      int64_t src[3][3];
      int xsl[3];
      source_rows<9>(d, y, 0, src);
      source_x(d, x, xsl);
      store_ghosts<9, ST>(d, fout, inf, src, xsl, f0, f1);
    }
  }
}

// ---------------------------------------------------------------------------
// D3Q19 fused step.  A block owns a 60 x kTileY3 column of (x, y) and marches
// through a chunk of z.  Per plane it keeps densities of the 64 x (kTileY3+4)
// region in an LDS ring of five planes (z-2 .. z+2): at plane z it forms rho of
// plane z+2, psi at the solid nodes of plane z+1, and collides plane z.  The
// interior populations of plane z are pulled again for the collision (they
// were fetched two planes earlier and come from cache), which keeps the
// register footprint small.  Wave w owns interior rows 2+w and 6+w and one
// halo row; rows and planes are wave-uniform.
// ---------------------------------------------------------------------------
constexpr int kRH3 = kTileY3 + 4;
constexpr int kRing = 5;

__device__ __forceinline__ int ring(int z) { return ((z % kRing) + kRing) % kRing; }

template <int COLL, int ST, typename R>
__global__ __launch_bounds__(256) void step_d3q19(const InstDev *__restrict__ insts,
                                                   const int32_t *__restrict__ block_inst, int parity) {
  using L = Lat<19>;
  using V = Vec2<R>;
  __shared__ V psi[kRing][kRH3][64];

  const int bid = xcd_block();
  const int inst = __builtin_amdgcn_readfirstlane(block_inst ? block_inst[bid] : 0);
  const InstDev &d = insts[inst];
  const int lb = bid - d.block_base;
  const int tx = lb % d.tiles_x, ty = (lb / d.tiles_x) % d.tiles_y;
  const int zc = lb / (d.tiles_x * d.tiles_y);  // z chunk
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  gcf *__restrict__ fin = G(d.f[parity]);
  gf *__restrict__ fout = G(d.f[parity ^ 1]);
  gcu32 *__restrict__ infop = (gcu32 *)d.info;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const bool px = d.periodic & 1, py = d.periodic & 2, pz = d.periodic & 4;
  const int zlen = (nz + d.tiles_z - 1) / d.tiles_z;
  const int z0 = zc * zlen, z1 = min(nz, z0 + zlen);
  const int64_t islab = (int64_t)d.pitch * ny;

  int gx = tx * kTileX - 2 + lane;
  const bool col_store = lane >= 2 && lane < 62 && gx < nx;
  bool col_in = true;
  if (gx < 0 || gx >= nx) {
    if (px) gx = wrap_index(gx, nx);
    else col_in = false;
  }
  const int gxa = col_in ? gx : (gx < 0 ? 0 : nx - 1);
  int xs[3];
  source_x(d, gxa, xs);
  // rows of this wave (uniform): interior rows 2+w, 6+w (k = 0, 1) and a halo row (k = 2)
  int rows[3], gy[3], gy_raw[3];
  bool row_in[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    rows[k] = k < 2 ? 2 + wave + 4 * k : (wave < 2 ? wave : kTileY3 + wave);
    int y = ty * kTileY3 - 2 + rows[k];
    gy_raw[k] = y;
    bool in = true;
    if (y < 0 || y >= ny) {
      if (py) y = wrap_index(y, ny);
      else in = false;
    }
    gy[k] = in ? y : 0;
    row_in[k] = in;
  }

  // plane index with periodic wrap; false if outside a closed z edge
  auto wrap_z = [&](int zp, int &zz) __attribute__((always_inline)) -> bool {
    zz = zp;
    if (zz < 0 || zz >= nz) {
      if (pz) { zz = wrap_index(zz, nz); return true; }
      zz = 0;
      return false;
    }
    return true;
  };

  // densities of the region rows of plane zp -> LDS ring
  auto load_plane = [&](int zp) __attribute__((always_inline)) {
    const int slot = ring(zp);
    int zz;
    const bool zin = wrap_z(zp, zz);
    uint32_t inf[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      inf[k] = (row_in[k] && col_in && zin) ? infop[gx + (int64_t)d.pitch * gy[k] + islab * zz] : kSolid;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R rho1 = 0, rho2 = 0;
      if (!(inf[k] & kSolid)) {
        int64_t src[3][3];
        source_rows<19, true>(d, gy[k], zz, src);
        float a[19], b[19];
        pull_row<19, ST>(d, fin, inf[k], src, xs, a, b);
        if (inf[k] & (kInlet | kOutlet)) complete<19, ST, R>(d, fin, inf[k], gx, gy[k], zz, a, b);
        rho1 = sum_q<19, R>(a);
        rho2 = sum_q<19, R>(b);
      }
      psi[slot][rows[k]][lane] = V{rho1, rho2};
    }
  };

  // virtual solid density (Eq. 17) at the solid nodes of plane zp, in place;
  // reads rho at planes zp-1 .. zp+1
  auto solid_psi = [&](int zp) __attribute__((always_inline)) {
    const int slot = ring(zp);
    int zz;
    if (!wrap_z(zp, zz)) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int r = rows[k];
      if (!row_in[k] || !col_in || r < 1 || r > kRH3 - 2 || lane < 1 || lane > 62) continue;
      const uint32_t nb = infop[gx + (int64_t)d.pitch * gy[k] + islab * zz];
      if (!(nb & kSolid) || !(nb & kLinkMask)) continue;
      if (d.ivsd0) {  // frozen reading of Eq. 17: the held value
        const v2f h = ivsd_held(d, gx + (int64_t)d.pitch * gy[k] + islab * zz);
        psi[slot][r][lane] = V{(R)h.x, (R)h.y};
        continue;
      }
      R s1 = 0, s2 = 0, den = 0;
#pragma unroll
      for (int i = 1; i < 19; ++i) {
        if (nb & (1u << i)) {
          const V p = psi[ring(zp + L::ez[i])][r + L::ey[i]][lane + L::ex[i]];
          const R w = (R)L::w[i];
          s1 += w * p.x;
          s2 += w * p.y;
          den += w;
        }
      }
      const R inv = rcp<R>(den);
      psi[slot][r][lane] = V{(R)d.chi1 * s1 * inv, (R)d.chi2 * s2 * inv};
    }
  };

  // force (Eq. 13 with the open-face mirror) + collision + store, plane z
  auto collide_plane = [&](int z) __attribute__((always_inline)) {
#pragma unroll 1
    for (int k = 0; k < 2; ++k) {
      if (!col_store || !row_in[k] || gy_raw[k] >= ny) continue;
      const int ri = rows[k];
      const uint32_t inf = infop[gx + (int64_t)d.pitch * gy[k] + islab * z];
      if (inf & kSolid) continue;
      int64_t src[3][3];
      source_rows<19, true>(d, gy[k], z, src);
      float a[19], b[19];
      pull_row<19, ST>(d, fin, inf, src, xs, a, b);
      if (inf & (kInlet | kOutlet)) complete<19, ST, R>(d, fin, inf, gx, gy[k], z, a, b);
      const V c = psi[ring(z)][ri][lane];
      const R rho1 = c.x, rho2 = c.y;
      R sx1 = 0, sy1 = 0, sz1 = 0, sx2 = 0, sy2 = 0, sz2 = 0;
      const bool open_face = (inf & (kInlet | kOutlet)) != 0;
#pragma unroll
      for (int i = 1; i < 19; ++i) {
        if (L::opp[i] < i) continue;
        const int o = L::opp[i];
        if (open_face && L::ex[i] != 0) continue;  // mirrored pair cancels
        const V pa = psi[ring(z + L::ez[i])][ri + L::ey[i]][lane + L::ex[i]];
        const V pb = psi[ring(z + L::ez[o])][ri + L::ey[o]][lane + L::ex[o]];
        const R w = (R)L::w[i];
        const R d1 = w * (pa.x - pb.x), d2 = w * (pa.y - pb.y);
        if (L::ex[i]) { sx1 += L::ex[i] * d1; sx2 += L::ex[i] * d2; }
        if (L::ey[i]) { sy1 += L::ey[i] * d1; sy2 += L::ey[i] * d2; }
        if (L::ez[i]) { sz1 += L::ez[i] * d1; sz2 += L::ez[i] * d2; }
      }
      const R G_ = (R)d.G, gxb = (R)d.gx, gyb = (R)d.gy, gzb = (R)d.gz;
      collide_node<19, COLL, R>(d, a, b, rho1, rho2, -G_ * rho1 * sx2 + rho1 * gxb,
                                -G_ * rho1 * sy2 + rho1 * gyb, -G_ * rho1 * sz2 + rho1 * gzb,
                                -G_ * rho2 * sx1 + rho2 * gxb, -G_ * rho2 * sy1 + rho2 * gyb,
                                -G_ * rho2 * sz1 + rho2 * gzb);
      pop_store<19, ST>(fout, d.pitch, uniform64(gy_raw[k] * d.ystride + z * d.zstride), gx, a, b, (float)rho1,
                        (float)rho2);
      store_ghosts<19, ST>(d, fout, inf, src, xs, a, b);
    }
  };

  // prologue: densities of planes z0-2 .. z0+1, psi of planes z0-1 and z0
  for (int zp = z0 - 2; zp <= z0 + 1; ++zp) load_plane(zp);
  __syncthreads();
  solid_psi(z0 - 1);
  solid_psi(z0);
  __syncthreads();
  for (int z = z0; z < z1; ++z) {
    load_plane(z + 2);
    __syncthreads();
    solid_psi(z + 1);  // needs rho at z .. z+2
    __syncthreads();
    collide_plane(z);
    // ring slot of z-2 is rewritten at z+3: every read of it is behind this barrier
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The pseudopotential between the launches of a step: (psi1, psi2) FP32
// pairs in the psi buffer.  Array 0 is dense, index x + pitch * (y + ny * z)
// like the node info: the densities at fluid nodes (split step) and the
// virtual solid density of Eq. 17 at solid nodes next to fluid.  Array 1
// holds, for the compacted split step, the fluid densities by compact index
// (the compacted 3D fused step uses both arrays as its carried psi, one per
// buffer parity).
// ---------------------------------------------------------------------------
__device__ __forceinline__ gv2f *psi32(const InstDev &d, int p) {
  return (gv2f *)d.psi + (int64_t)p * d.pitch * d.ny * d.nz;
}

__device__ __forceinline__ int wrap3(int p) { return ((p % 3) + 3) % 3; }

// Pair sums sum_i w_i psi(x + e_i) e_i of Eq. 13 from the eighteen (or
// eight) neighbour values pv[i] = psi(x + e_i); at an open face the mirrored
// pairs with an x component cancel.
template <int Q, typename R>
__device__ __forceinline__ void force_sums(const v2f (&pv)[Q], bool open_face, R &sx1, R &sy1, R &sz1, R &sx2,
                                           R &sy2, R &sz2) {
  using L = Lat<Q>;
  sx1 = 0; sy1 = 0; sz1 = 0; sx2 = 0; sy2 = 0; sz2 = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (L::opp[i] < i) continue;
    const int o = L::opp[i];
    const v2f pa = pv[i], pb = pv[o];
    const R w = (R)L::w[i];
    R d1 = w * ((R)pa.x - (R)pb.x), d2 = w * ((R)pa.y - (R)pb.y);
    if (L::ex[i] != 0) {
      d1 = open_face ? R(0) : d1;
      d2 = open_face ? R(0) : d2;
    }
    if (L::ex[i]) { sx1 += L::ex[i] * d1; sx2 += L::ex[i] * d2; }
    if (L::ey[i]) { sy1 += L::ey[i] * d1; sy2 += L::ey[i] * d2; }
    if (L::ez[i]) { sz1 += L::ez[i] * d1; sz2 += L::ez[i] * d2; }
  }
}

// The neighbour values pv[i] = psi(x + e_i) from a dense psi array: every
// neighbour is loaded, with no branch between the loads, so they are all in
// flight at once (an open face drops the mirrored x pairs afterwards).
template <int Q>
__device__ __forceinline__ void psi32_neighbours(const InstDev &d, gcv2f *__restrict__ psi, int x, int y, int z,
                                                 v2f (&pv)[Q]) {
  using L = Lat<Q>;
  int xs[3];
  source_x(d, x, xs);  // xs[1 - e_x]: x + e_x with wrap
  const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? d.nz - 1 : z - 1, zp = z == d.nz - 1 ? 0 : z + 1;
  const uint32_t pitch = (uint32_t)d.pitch, ny = (uint32_t)d.ny;
  const uint32_t yy[3] = {(uint32_t)ym, (uint32_t)y, (uint32_t)yp}, zz[3] = {(uint32_t)zm, (uint32_t)z, (uint32_t)zp};
  pv[0] = v2f{0.f, 0.f};
#pragma unroll
  for (int i = 1; i < Q; ++i)
    pv[i] = psi[(uint32_t)xs[1 - L::ex[i]] + pitch * (yy[L::ey[i] + 1] + ny * zz[L::ez[i] + 1])];
}

// Pair sums of Eq. 13 from a dense psi array.
template <int Q, typename R>
__device__ __forceinline__ void psi32_force_sums(const InstDev &d, gcv2f *__restrict__ psi, int x, int y, int z,
                                                 bool open_face, R &sx1, R &sy1, R &sz1, R &sx2, R &sy2,
                                                 R &sz2) {
  v2f pv[Q];
  psi32_neighbours<Q>(d, psi, x, y, z, pv);
  force_sums<Q, R>(pv, open_face, sx1, sy1, sz1, sx2, sy2, sz2);
}

// ---------------------------------------------------------------------------
// Split step (three launches) for grids whose per-block working set does not
// fit the L2: the halo recompute of the fused kernels would then refetch
// populations from memory.  Each wave owns 64 consecutive x of one (y, z)
// row (wave-uniform rows), one thread per node.
//   rho_kernel:     pull + complete -> rho^s(x) into dense psi array 0 (FP32)
//   psi_kernel:     virtual solid density (Eq. 17) at solid nodes, in place
//   collide_kernel: force from psi (Eq. 13 with the open-face mirror), pull
//                   again, densities from the pull, collide, store
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool wave_row(const InstDev &d, int &x, int &y, int &z) {
  const int segs = (d.nx + 63) >> 6;
  const int64_t W = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t row = W / segs;
  const int seg = (int)(W - row * segs);
  y = (int)(row % d.ny);
  z = (int)(row / d.ny);
  x = seg * 64 + (int)(threadIdx.x & 63);
  return z < d.nz && x < d.nx;
}

template <int Q, int ST>
__global__ __launch_bounds__(256) void rho_kernel(const InstDev *__restrict__ insts, int parity) {
  const InstDev &d = insts[0];
  int x, y, z;
  if (!wave_row(d, x, y, z)) return;
  const int64_t pi = x + (int64_t)d.pitch * (y + (int64_t)d.ny * z);
  const uint32_t info = ((gcu32 *)d.info)[pi];
  if (info & kSolid) return;
  gcf *__restrict__ fin = G(d.f[parity]);
  int64_t src[3][3];
  int xs[3];
  source_rows<Q, true>(d, y, z, src);  // one row per wave
  source_x(d, x, xs);
  float a[Q], b[Q];
  pull_row<Q, ST>(d, fin, info, src, xs, a, b);
  if (info & (kInlet | kOutlet)) complete<Q, ST, double>(d, fin, info, x, y, z, a, b);
  psi32(d, 0)[pi] = v2f{(float)sum_q<Q, double>(a), (float)sum_q<Q, double>(b)};
}

// Virtual solid density (Eq. 17) of solid node (x, y, z), whose fluid
// neighbours are flagged in nb; fluid density of neighbour (xn, yn, zn) from
// dens(xn, yn, zn), summed in FP64.
template <int Q, class DensF>
__device__ __forceinline__ v2f ivsd_value(const InstDev &d, int x, int y, int z, uint32_t nb, DensF dens) {
  using L = Lat<Q>;
  int xs[3];
  source_x(d, x, xs);  // xs[1 - e_x]: x + e_x with wrap
  const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? d.nz - 1 : z - 1, zp = z == d.nz - 1 ? 0 : z + 1;
  const int yy[3] = {ym, y, yp}, zz[3] = {zm, z, zp};  // index by e + 1
  double s1 = 0, s2 = 0, den = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (nb & (1u << i)) {
      const v2f p = dens(xs[1 - L::ex[i]], yy[L::ey[i] + 1], zz[L::ez[i] + 1]);
      s1 += L::w[i] * (double)p.x;
      s2 += L::w[i] * (double)p.y;
      den += L::w[i];
    }
  }
  const double inv = rcp<double>(den);
  return v2f{(float)(d.chi1 * s1 * inv), (float)(d.chi2 * s2 * inv)};
}

// Eq. 17 at solid node (x, y, z), dense index pi, into dense psi array 0
// (the held value under the frozen reading).
template <int Q, class DensF>
__device__ __forceinline__ void ivsd_node(const InstDev &d, int x, int y, int z, int64_t pi, uint32_t nb,
                                          DensF dens) {
  psi32(d, 0)[pi] = d.ivsd0 ? ivsd_held(d, pi) : ivsd_value<Q>(d, x, y, z, nb, dens);
}

template <int Q>
__global__ __launch_bounds__(256) void psi_kernel(const InstDev *__restrict__ insts) {
  const InstDev &d = insts[0];
  int x, y, z;
  if (!wave_row(d, x, y, z)) return;
  const int64_t pi = x + (int64_t)d.pitch * (y + (int64_t)d.ny * z);
  const uint32_t nb = ((gcu32 *)d.info)[pi];
  if (!(nb & kSolid) || !(nb & kLinkMask)) return;
  gcv2f *__restrict__ psi = psi32(d, 0);
  ivsd_node<Q>(d, x, y, z, pi, nb, [&](int xn, int yn, int zn) {
    return psi[xn + (int64_t)d.pitch * (yn + (int64_t)d.ny * zn)];
  });
}

template <int Q, int COLL, int ST, typename R>
__global__ __launch_bounds__(256) void collide_kernel(const InstDev *__restrict__ insts, int parity) {
  const InstDev &d = insts[0];
  int x, y, z;
  if (!wave_row(d, x, y, z)) return;
  const int64_t pi = x + (int64_t)d.pitch * (y + (int64_t)d.ny * z);
  const uint32_t info = ((gcu32 *)d.info)[pi];
  if (info & kSolid) return;
  gcf *__restrict__ fin = G(d.f[parity]);
  gf *__restrict__ fout = G(d.f[parity ^ 1]);
  int xs[3];
  source_x(d, x, xs);
  R sx1, sy1, sz1, sx2, sy2, sz2;
  psi32_force_sums<Q, R>(d, psi32(d, 0), x, y, z, (info & (kInlet | kOutlet)) != 0, sx1, sy1, sz1, sx2, sy2, sz2);
  // keep the psi loads and the pulls apart (register pressure)
  __builtin_amdgcn_sched_barrier(0);
  int64_t src[3][3];
  source_rows<Q, true>(d, y, z, src);  // one row per wave
  float a[Q], b[Q];
  pull_row<Q, ST>(d, fin, info, src, xs, a, b);
  if (info & (kInlet | kOutlet)) complete<Q, ST, R>(d, fin, info, x, y, z, a, b);
  const R rho1 = sum_q<Q, R>(a), rho2 = sum_q<Q, R>(b);
  const R G_ = (R)d.G, gxb = (R)d.gx, gyb = (R)d.gy, gzb = (R)d.gz;
  collide_node<Q, COLL, R>(d, a, b, rho1, rho2, -G_ * rho1 * sx2 + rho1 * gxb, -G_ * rho1 * sy2 + rho1 * gyb,
                           -G_ * rho1 * sz2 + rho1 * gzb, -G_ * rho2 * sx1 + rho2 * gxb,
                           -G_ * rho2 * sy1 + rho2 * gyb, -G_ * rho2 * sz1 + rho2 * gzb);
  pop_store<Q, ST, Q == 19>(fout, d.pitch, uniform64(y * d.ystride + z * d.zstride), x, a, b, (float)rho1,
                           (float)rho2);
  store_ghosts<Q, ST>(d, fout, info, src, xs, a, b);
}

// ---------------------------------------------------------------------------
// Compacted fluid-node step.  Thread per fluid node (nothing is spent on solid
// nodes, whose populations are not stored).  The state is f*[s][i][c] over
// the compact index c; a pull from a fluid source reads the source's compact
// index (popcount rank in its row), a pull across a solid link reads the
// node's own f*_opp(i) (half-way bounce-back without ghost slots).  Densities
// and the virtual solid density go through dense psi array 0 as in the split
// step, and the force and collision are the split step's arithmetic.
// ---------------------------------------------------------------------------

// Does some link of the lattice pull from row offset (dy, dz)?
template <int Q>
__device__ __forceinline__ constexpr bool row_used(int dy, int dz) {
  for (int i = 1; i < Q; ++i)
    if (Lat<Q>::ey[i] == dy && Lat<Q>::ez[i] == dz) return true;
  return false;
}

__device__ __forceinline__ void ckey_xyz(const InstDev &d, uint32_t key, int &x, int &y, int &z) {
  const uint32_t r = key / (uint32_t)d.pitch;
  x = (int)(key - r * (uint32_t)d.pitch);
  y = (int)(r % (uint32_t)d.ny);
  z = (int)(r / (uint32_t)d.ny);
}

// Compact index scs[i] of the pull source x - e_i of every link of fluid node
// c at (x, y, z) (scs[0] = c).  A link whose source is solid gets a value
// that is never used (bounce-back reads the node's own slot); a link across
// an open face gets the periodic image's, overwritten by the completion.
// The host keeps compact indices below 2^32.
template <int Q>
__device__ __forceinline__ void csources(const InstDev &d, int x, int y, int z, int64_t c, uint32_t (&scs)[Q]) {
  using L = Lat<Q>;
  int xs[3];
  source_x(d, x, xs);  // indexed by e_x + 1: x - e_x with wrap
  const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? d.nz - 1 : z - 1, zp = z == d.nz - 1 ? 0 : z + 1;
  const int ys[3] = {yp, y, ym}, zs[3] = {zp, z, zm};  // indexed by e + 1: y - e_y, z - e_z
  const int64_t last = d.nf - 1;
  // Rank rk and fluid bit fl at column x of every source row (one row word
  // each; the node's own row is rk = c, fl = 1).  A fluid source at x - 1 has
  // rank rk - 1, one at x + 1 rank rk + fl (a row's fluid nodes are numbered
  // consecutively); sources across the x edge are looked up.
  uint32_t rk[3][3], fl[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      rk[a][b] = (uint32_t)c;
      fl[a][b] = 1;
      if ((a == 1 && b == 1) || !row_used<Q>(a - 1, b - 1)) continue;
      const int64_t row = ys[a] + (int64_t)d.ny * zs[b];
      const RowWord w = row_word(d, row * (d.pitch >> 6) + (x >> 6));
      rk[a][b] = (uint32_t)(w.pre + __popcll(w.bits & ((1ull << (x & 63)) - 1ull)));
      fl[a][b] = (uint32_t)((w.bits >> (x & 63)) & 1ull);
    }
  scs[0] = (uint32_t)c;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int a = L::ey[i] + 1, b = L::ez[i] + 1;
    scs[i] = L::ex[i] == 0 ? rk[a][b] : (L::ex[i] > 0 ? rk[a][b] - 1 : rk[a][b] + fl[a][b]);
  }
  const bool cross_lo = x == 0, cross_hi = x == d.nx - 1;
  if (cross_lo || cross_hi) {
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if ((L::ex[i] > 0 && cross_lo) || (L::ex[i] < 0 && cross_hi)) {
        const int64_t k = crank(d, xs[L::ex[i] + 1], ys[L::ey[i] + 1] + (int64_t)d.ny * zs[L::ez[i] + 1]);
        scs[i] = (uint32_t)(k < last ? k : last);
      }
    }
  }
}

// Pull of fluid node c from the sources scs (bounce-back across solid links)
// + inlet/outlet completion.
template <int Q, int ST, typename R>
__device__ __forceinline__ void cpull(const InstDev &d, gcf *__restrict__ fin, uint32_t info, int y, int z,
                                      int64_t c, const uint32_t (&scs)[Q], float (&f0)[Q], float (&f1)[Q]) {
  using L = Lat<Q>;
  const int cp = d.cpitch;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const bool bb = i != 0 && ((info >> i) & 1u);  // half-way bounce-back: own opposite slot
    const int pi = bb ? L::opp[i] : i;
    const uint32_t sc = bb ? (uint32_t)c : scs[i];
    if constexpr (ST == 0) {
      // component regions from a wave-uniform base, 32-bit byte offsets
      const uint32_t bo = cslot<Q>(sc, pi) * 4u;
      f0[i] = ldg(fin, bo);
      f1[i] = ldg(fin + (int64_t)Q * cp, bo);
    } else {
      pop_get2<Q, ST>(fin, cp, pi, 0, (int)sc, f0[i], f1[i]);
    }
  }
  if (info & (kInlet | kOutlet)) {
    const int t = y + d.ny * z;
    const int64_t nt = (int64_t)d.ny * d.nz;
    gcf *frz = G(d.frozen);
    complete_boundary<Q, R>(
        d, info, f0, f1, [&](int s, int i) { return cpop_get<Q, ST>(fin, cp, s, i, c); },
        [&](int s, int i) { return frz[(int64_t)(s * Q + i) * nt + t]; });
  }
}

// Pull + inlet/outlet completion of fluid node c at (x, y, z).
template <int Q, int ST, typename R>
__device__ __forceinline__ void cgather(const InstDev &d, gcf *__restrict__ fin, uint32_t info, int x, int y,
                                        int z, int64_t c, float (&f0)[Q], float (&f1)[Q]) {
  uint32_t scs[Q];
  csources<Q>(d, x, y, z, c, scs);
  cpull<Q, ST, R>(d, fin, info, y, z, c, scs, f0, f1);
}

template <int Q, int ST>
__global__ __launch_bounds__(256) void crho_kernel(const InstDev *__restrict__ insts, int parity) {
  const InstDev &d = insts[0];
  const int64_t c = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
  if (c >= d.nf) return;
  const uint32_t key = gld32(d.ckey, c);
  int x, y, z;
  ckey_xyz(d, key, x, y, z);
  const uint32_t info = gld32(d.cinfo, c);
  float a[Q], b[Q];
  cgather<Q, ST, double>(d, G(d.f[parity]), info, x, y, z, c, a, b);
  psi32(d, 0)[key] = v2f{(float)sum_q<Q, double>(a), (float)sum_q<Q, double>(b)};
}

template <int Q>
__global__ __launch_bounds__(256) void cpsi_kernel(const InstDev *__restrict__ insts) {
  const InstDev &d = insts[0];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.nbnd) return;
  const uint32_t key = gld32(d.cbnd, j);
  int x, y, z;
  ckey_xyz(d, key, x, y, z);
  gcv2f *__restrict__ psi = psi32(d, 0);
  ivsd_node<Q>(d, x, y, z, key, ((gcu32 *)d.info)[key], [&](int xn, int yn, int zn) {
    return psi[xn + (int64_t)d.pitch * (yn + (int64_t)d.ny * zn)];
  });
}

template <int Q, int COLL, int ST, typename R>
__global__ __launch_bounds__(256) void ccollide_kernel(const InstDev *__restrict__ insts, int parity) {
  const InstDev &d = insts[0];
  const int64_t c = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
  if (c >= d.nf) return;
  const uint32_t key = gld32(d.ckey, c);
  int x, y, z;
  ckey_xyz(d, key, x, y, z);
  const uint32_t info = gld32(d.cinfo, c);
  // the neighbours' psi and the source ranks' row words depend only on the
  // node's position: both are in flight in one round trip
  v2f pv[Q];
  psi32_neighbours<Q>(d, psi32(d, 0), x, y, z, pv);
  uint32_t scs[Q];
  csources<Q>(d, x, y, z, c, scs);
  R sx1, sy1, sz1, sx2, sy2, sz2;
  force_sums<Q, R>(pv, (info & (kInlet | kOutlet)) != 0, sx1, sy1, sz1, sx2, sy2, sz2);
  // keep the psi loads and the pulls apart: both in flight at once would
  // double the live registers and halve the waves per SIMD
  __builtin_amdgcn_sched_barrier(0);
  float a[Q], b[Q];
  cpull<Q, ST, R>(d, G(d.f[parity]), info, y, z, c, scs, a, b);
  const R rho1 = sum_q<Q, R>(a), rho2 = sum_q<Q, R>(b);
  const R G_ = (R)d.G, gxb = (R)d.gx, gyb = (R)d.gy, gzb = (R)d.gz;
  collide_node<Q, COLL, R>(d, a, b, rho1, rho2, -G_ * rho1 * sx2 + rho1 * gxb, -G_ * rho1 * sy2 + rho1 * gyb,
                           -G_ * rho1 * sz2 + rho1 * gzb, -G_ * rho2 * sx1 + rho2 * gxb,
                           -G_ * rho2 * sy1 + rho2 * gyb, -G_ * rho2 * sz1 + rho2 * gzb);
  cpop_store<Q, ST, Q == 19>(G(d.f[parity ^ 1]), d.cpitch, c, a, b, (float)rho1, (float)rho2);
}

// ---------------------------------------------------------------------------
// D3Q19 fused step over the compacted layout with FP32 storage
// (LBM_COMPACT_FUSED for q = 19): every population is pulled once per step.
//
// Besides f*, the state between steps holds the pseudopotential the coming
// step needs (Eq. 13 with Eq. 15), as (psi1, psi2) float pairs on the dense
// grid: rho^s(x, t+1) = sum_i f^s_i(x, t+1) at fluid nodes and the virtual
// solid density of Eq. 17 at solid nodes next to fluid.  Two such arrays fill
// the psi buffer and alternate with the population buffers.  A step is three
// launches:
//   fwd_step_d3q19   a block owns a tile of one row word (64 columns) by
//                    kFwdRows rows and marches a chunk of z.  Per plane it
//                    lists the tile's fluid nodes; one thread per list entry
//                    pulls the node's populations, forms its densities,
//                    reads the neighbours' psi from the carried array,
//                    collides, stores f* and stages it in LDS.  Each tile
//                    position then adds up what its fluid sources in the
//                    tile stream into it (bounce-back and rest links come
//                    from the node itself), so rho(t+1) is complete, and
//                    written, at every node whose 18 sources lie in the tile
//                    and chunk: all but the tile's outer ring and the
//                    chunk's end planes.
//   fwd_rho_kernel   those edge nodes pull their t+1 populations from the new
//                    f* and sum them, as the compacted density kernel does
//                    (every fluid node when the carried array is rebuilt).
//   fwd_ivsd_kernel  Eq. 17 at the solid nodes next to fluid.
// The node arithmetic is the compacted split step's; psi is carried in FP32.
// ---------------------------------------------------------------------------
constexpr int kFwdThreads = 256;             // list entries collided per round
constexpr int kFwdPos = 64 * kFwdRows;       // tile positions per plane

// Block barrier for LDS traffic only: waits for the wave's own LDS (and
// scalar) operations, not for its global loads and stores, which no other
// thread of the launch reads.  (__syncthreads would also drain every
// outstanding global store at each plane's barriers.)
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int COLL, typename R>
__global__ __launch_bounds__(kFwdThreads) __attribute__((amdgpu_waves_per_eu(3))) void fwd_step_d3q19(
    const InstDev *__restrict__ insts, const int32_t *__restrict__ block_inst, int parity) {
  using L = Lat<19>;
  constexpr int Q = 19;
  constexpr int RW = kFwdRows + 2;  // staged rows: y0 - 1 .. y0 + kFwdRows
  constexpr int RC = 66;            // rank columns: x0 - 1 .. x0 + 64
  // compact index of the node at each staged (plane mod 3, row, column)
  // when it is fluid
  __shared__ int32_t rtab[3][RW][RC];
  __shared__ unsigned long long fbits[3][kFwdRows];  // fluid bits of the tile rows
  __shared__ uint16_t lst[2][kFwdPos];               // (row << 6) | column, by plane parity
  __shared__ int nls[2];
  // one component's post-collision links of the round's nodes by tile
  // position; link 0 holds the node's own share of its next density (rest
  // link and bounced links); positions without a node of the round hold 0
  __shared__ float stage[Q][kFwdPos];

  const int bid = xcd_block();
  const int inst = __builtin_amdgcn_readfirstlane(block_inst ? block_inst[bid] : 0);
  const InstDev &d = insts[inst];
  const int lb = bid - d.block_base;
  const int tx = lb % d.tiles_x, ty = (lb / d.tiles_x) % d.tiles_y;
  const int zc = lb / (d.tiles_x * d.tiles_y);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int zlen = (nz + d.tiles_z - 1) / d.tiles_z;
  const int z0 = zc * zlen, z1 = min(nz, z0 + zlen);
  if (z0 >= z1) return;  // the whole block
  const int x0 = tx * 64, y0 = ty * kFwdRows;
  const int W = min(64, nx - x0), H = min(kFwdRows, ny - y0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t wpr = d.pitch >> 6;
  const uint32_t cp = (uint32_t)d.cpitch, pitch = (uint32_t)d.pitch;
  const bool py = d.periodic & 2, pz = d.periodic & 4;
  const bool open_x = d.open_x != 0;
  gcf *__restrict__ fin = G(d.f[parity]);
  gf *__restrict__ fout = G(d.f[parity ^ 1]);
  gcf *__restrict__ frz = G(d.frozen);
  gcv2f *__restrict__ psi_in = psi32(d, parity);
  gv2f *__restrict__ psi_out = psi32(d, parity ^ 1);
  const R G_ = (R)d.G, gxb = (R)d.gx, gyb = (R)d.gy, gzb = (R)d.gz;

  // staged row words of plane p (rows y0 - 1 .. y0 + kFwdRows; rows outside
  // a closed y or z edge hold no fluid), read with scalar loads, which wait
  // on no vector load or store of the wave; the tile rows' fluid bits too
  // (with the words left and right of the tile's, for the first and last column)
  __shared__ RowWord wst[RW][3];
  auto stage_words = [&](int p) __attribute__((always_inline)) {
    for (int k = wave; k < RW; k += kFwdThreads / 64) {
      int yy = y0 - 1 + k, zz = p;
      bool in = true;
      if (yy < 0 || yy >= ny) { if (py) yy = wrap_index(yy, ny); else in = false; }
      if (zz < 0 || zz >= nz) { if (pz) zz = wrap_index(zz, nz); else in = false; }
      RowWord w[3];
#pragma unroll
      for (int h = 0; h < 3; ++h) {
        w[h] = RowWord{0ull, 0ll};
        const int t = tx - 1 + h;
        if (in && t >= 0 && t < wpr) {
          const int64_t wi = ((int64_t)yy + (int64_t)ny * zz) * wpr + t;
          typedef __attribute__((address_space(4))) const RowWord kRowWord;
          const kRowWord *cw = (const kRowWord *)d.cword + uniform64(wi);
          w[h].bits = cw->bits;
          w[h].pre = cw->pre;
        }
      }
      if (lane == 0) { wst[k][0] = w[0]; wst[k][1] = w[1]; wst[k][2] = w[2]; }
      if (lane == 0 && k >= 1 && k <= kFwdRows) fbits[wrap3(p)][k - 1] = k - 1 < H ? w[1].bits : 0ull;
    }
  };
  // rank table of plane p and its fluid list (after put_words(p) and a barrier)
  auto build_plane = [&](int p) __attribute__((always_inline)) {
    const int s = wrap3(p);
    for (int e = tid; e < RW * RC; e += kFwdThreads) {
      const int k = e / RC, c = e - k * RC;
      int32_t v;
      if (c == 0) {  // x0 - 1: the last column of the word on the left
        const RowWord w = wst[k][0];
        v = (int32_t)(w.pre + __popcll(w.bits & ((1ull << 63) - 1ull)));
      } else if (c == RC - 1) {  // x0 + 64: the first column of the word on the right
        v = (int32_t)wst[k][2].pre;
      } else {
        const RowWord w = wst[k][1];
        v = (int32_t)(w.pre + __popcll(w.bits & ((1ull << (c - 1)) - 1ull)));
      }
      rtab[s][k][c] = v;
    }
    // wave w lists rows w and w + 4
#pragma unroll
    for (int j = 0; j < kFwdRows / 4; ++j) {
      const int r = wave + 4 * j;
      int pre = 0;
#pragma unroll
      for (int rr = 0; rr < kFwdRows; ++rr)
        if (rr < r && rr < H) pre += __popcll(wst[rr + 1][1].bits);
      const unsigned long long bits = r < H ? wst[r + 1][1].bits : 0ull;
      if ((bits >> lane) & 1ull) lst[p & 1][pre + __popcll(bits & ((1ull << lane) - 1ull))] = (uint16_t)((r << 6) | lane);
    }
    if (tid == 0) {
      int total = 0;
#pragma unroll
      for (int rr = 0; rr < kFwdRows; ++rr)
        if (rr < H) total += __popcll(wst[rr + 1][1].bits);
      nls[p & 1] = total;
    }
  };

  stage_words(z0 - 1);
  lds_barrier();
  build_plane(z0 - 1);
  lds_barrier();
  stage_words(z0);
  lds_barrier();
  build_plane(z0);
  // next-step density sums of this thread's positions (rows wave and
  // wave + 4, column lane) on planes z - 1, z, z + 1
  float acc[2][3][2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[j][k][0] = acc[j][k][1] = 0.f;

  for (int z = z0; z < z1; ++z) {
    lds_barrier();  // the previous plane's rank tables are read
    stage_words(z + 1);
    lds_barrier();
    build_plane(z + 1);
    lds_barrier();
    const int n = nls[z & 1];
    const int sz = wrap3(z);
    for (int base = 0; base < n; base += kFwdThreads) {
      // positions without a node of this round stream nothing
#pragma unroll
      for (int i = 0; i < Q; ++i)
        for (int e = tid; e < kFwdPos; e += kFwdThreads) stage[i][e] = 0.f;
      const int e = base + tid;
      const bool act = e < n;
      int pos = 0;
      float a[Q], b[Q];
      if (act) {
        const int ent = lst[z & 1][e];
        const int r = ent >> 6, l = ent & 63;
        pos = ent;
        const int x = x0 + l, y = y0 + r;
        const uint32_t key = (uint32_t)x + pitch * ((uint32_t)y + (uint32_t)ny * (uint32_t)z);
        const bool face = open_x && (x == 0 || x == nx - 1);
        R sx1, sy1, sz1, sx2, sy2, sz2;
        psi32_force_sums<Q, R>(d, psi_in, x, y, z, face, sx1, sy1, sz1, sx2, sy2, sz2);
        const uint32_t info = ((gcu32 *)d.info)[key];
        // keep the psi loads and the pulls apart (register pressure)
        __builtin_amdgcn_sched_barrier(0);
        // compact index of every link's source from the rank tables (all read
        // before any pull is issued)
        const int sp[3] = {wrap3(z + 1), sz, wrap3(z - 1)};  // plane of z - e_z, by e_z + 1
        uint32_t sc[Q];
        sc[0] = (uint32_t)rtab[sz][r + 1][l + 1];
#pragma unroll
        for (int i = 1; i < Q; ++i) sc[i] = (uint32_t)rtab[sp[L::ez[i] + 1]][r - L::ey[i] + 1][l - L::ex[i] + 1];
        if (x == 0 || x == nx - 1) {
          // sources across the x edge: the periodic image, or a missing link at
          // an open face (any node; the completion below overwrites it)
#pragma unroll
          for (int i = 1; i < Q; ++i) {
            if ((L::ex[i] > 0 && x == 0) || (L::ex[i] < 0 && x == nx - 1)) {
              const int ys = wrap_index(y - L::ey[i], ny), zs = wrap_index(z - L::ez[i], nz);
              const int64_t k = crank(d, L::ex[i] > 0 ? nx - 1 : 0, ys + (int64_t)ny * zs);
              sc[i] = (uint32_t)(k < d.nf - 1 ? k : d.nf - 1);
            }
          }
        }
        const uint32_t c = sc[0];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          // half-way bounce-back: the node's own opposite slot
          const bool bb = i != 0 && ((info >> i) & 1u);
          const uint32_t pi = bb ? (uint32_t)L::opp[i] : (uint32_t)i;
          const uint32_t bo = cslot<Q>(bb ? c : sc[i], (int)pi) * 4u;
          a[i] = ldg(fin, bo);
          b[i] = ldg(fin + (int64_t)Q * cp, bo);
        }
        if (face) {
          const int t = y + ny * z;
          const int64_t nt = (int64_t)ny * nz;
          complete_boundary<Q, R>(
              d, info, a, b, [&](int s_, int i) { return fin[(int64_t)s_ * Q * cp + cslot<Q>(c, i)]; },
              [&](int s_, int i) { return frz[(int64_t)(s_ * Q + i) * nt + t]; });
        }
        const R rho1 = sum_q<Q, R>(a), rho2 = sum_q<Q, R>(b);
        collide_node<Q, COLL, R>(d, a, b, rho1, rho2, -G_ * rho1 * sx2 + rho1 * gxb, -G_ * rho1 * sy2 + rho1 * gyb,
                                 -G_ * rho1 * sz2 + rho1 * gzb, -G_ * rho2 * sx1 + rho2 * gxb,
                                 -G_ * rho2 * sy1 + rho2 * gyb, -G_ * rho2 * sz1 + rho2 * gzb);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const uint32_t so = cslot<Q>(c, i) * 4u;
          stg(fout, so, a[i]);
          stg(fout + (int64_t)Q * cp, so, b[i]);
        }
        // the node's own share of its next density: rest link and the links
        // that bounce back into it
        float s1 = a[0], s2 = b[0];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const bool bb = (info >> i) & 1u;
          s1 += bb ? a[L::opp[i]] : 0.f;
          s2 += bb ? b[L::opp[i]] : 0.f;
        }
        a[0] = s1;
        b[0] = s2;
      }
      // one component at a time: stage by position, then every inner tile
      // position of planes z - 1, z, z + 1 adds what streams into it
#pragma unroll
      for (int comp = 0; comp < 2; ++comp) {
        lds_barrier();
        if (act) {
#pragma unroll
          for (int i = 0; i < Q; ++i) stage[i][pos] = comp ? b[i] : a[i];
        }
        lds_barrier();
#pragma unroll
        for (int j = 0; j < kFwdRows / 4; ++j) {
          const int r = wave + 4 * j;
          if (r < 1 || r > H - 2 || lane < 1 || lane > W - 2) continue;
          const int tp = (r << 6) | lane;
          float t0 = 0.f, t1 = stage[0][tp], t2 = 0.f;
#pragma unroll
          for (int i = 1; i < Q; ++i) {
            const float v = stage[i][tp - L::ex[i] - 64 * L::ey[i]];
            if (L::ez[i] < 0) t0 += v;
            else if (L::ez[i] == 0) t1 += v;
            else t2 += v;
          }
          acc[j][0][comp] += t0;
          acc[j][1][comp] += t1;
          acc[j][2][comp] += t2;
        }
      }
      lds_barrier();
    }
    // plane z - 1 has received all its links: its inner fluid nodes' densities
    const int pd = z - 1;
    if (pd > z0 && pd < z1 - 1) {
#pragma unroll
      for (int j = 0; j < kFwdRows / 4; ++j) {
        const int r = wave + 4 * j;
        if (r < 1 || r > H - 2 || lane < 1 || lane > W - 2 || !((fbits[wrap3(pd)][r] >> lane) & 1ull)) continue;
        const uint32_t key = (uint32_t)(x0 + lane) + pitch * ((uint32_t)(y0 + r) + (uint32_t)ny * (uint32_t)pd);
        psi_out[key] = v2f{acc[j][0][0], acc[j][0][1]};
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[j][0][0] = acc[j][1][0]; acc[j][0][1] = acc[j][1][1];
      acc[j][1][0] = acc[j][2][0]; acc[j][1][1] = acc[j][2][1];
      acc[j][2][0] = 0.f; acc[j][2][1] = 0.f;
    }
  }
}

// Densities of the coming step at the fluid nodes `list` names (every fluid
// node when list is NULL): pull from buffer `parity` with the inlet/outlet
// completion, sum, and store in carried psi array `parity`.
template <int Q>
__global__ __launch_bounds__(256) void fwd_rho_kernel(const InstDev *__restrict__ insts,
                                                      const uint32_t *__restrict__ list, int64_t n, int parity) {
  const InstDev &d = insts[0];
  const int64_t j = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t c = list ? (int64_t)gld32(list, j) : j;
  const uint32_t key = gld32(d.ckey, c);
  int x, y, z;
  ckey_xyz(d, key, x, y, z);
  const uint32_t info = gld32(d.cinfo, c);
  float a[Q], b[Q];
  cgather<Q, 0, double>(d, G(d.f[parity]), info, x, y, z, c, a, b);
  psi32(d, parity)[key] = v2f{(float)sum_q<Q, double>(a), (float)sum_q<Q, double>(b)};
}

// Virtual solid density (Eq. 17) at the solid nodes next to fluid, from the
// densities in carried psi array `parity`.
template <int Q>
__global__ __launch_bounds__(256) void fwd_ivsd_kernel(const InstDev *__restrict__ insts, int parity) {
  using L = Lat<Q>;
  const InstDev &d = insts[0];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.nbnd) return;
  const uint32_t key = gld32(d.cbnd, j);
  int x, y, z;
  ckey_xyz(d, key, x, y, z);
  const uint32_t nb = ((gcu32 *)d.info)[key];
  gv2f *__restrict__ psi = psi32(d, parity);
  if (d.ivsd0) {
    psi[key] = ivsd_held(d, key);
    return;
  }
  int xs[3];
  source_x(d, x, xs);  // xs[1 - e_x]: x + e_x with wrap
  const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? d.nz - 1 : z - 1, zp = z == d.nz - 1 ? 0 : z + 1;
  const int yy[3] = {ym, y, yp}, zz[3] = {zm, z, zp};
  double s1 = 0, s2 = 0, den = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (nb & (1u << i)) {
      const uint32_t k = (uint32_t)xs[1 - L::ex[i]] +
                         (uint32_t)d.pitch * ((uint32_t)yy[L::ey[i] + 1] + (uint32_t)d.ny * (uint32_t)zz[L::ez[i] + 1]);
      const v2f p = psi[k];
      s1 += L::w[i] * (double)p.x;
      s2 += L::w[i] * (double)p.y;
      den += L::w[i];
    }
  }
  const double inv = rcp<double>(den);
  psi[key] = v2f{(float)(d.chi1 * s1 * inv), (float)(d.chi2 * s2 * inv)};
}

template <int COLL, int ST, typename R>
static void launch_fused_q(int q, int ty, const InstDev *d, const int32_t *bi, int64_t nb, int parity,
                           hipStream_t s, bool compact = false) {
  const dim3 g((unsigned)nb), b(256);
  if (q == 9 && compact) {
    if (ty == 8) step_d2q9<COLL, ST, R, 8, 1><<<g, b, 0, s>>>(d, bi, parity);
    else if (ty == 16) step_d2q9<COLL, ST, R, 16, 1><<<g, b, 0, s>>>(d, bi, parity);
    else step_d2q9<COLL, ST, R, 12, 1><<<g, b, 0, s>>>(d, bi, parity);
  } else if (q == 9) {
    if (ty == 8) step_d2q9<COLL, ST, R, 8><<<g, b, 0, s>>>(d, bi, parity);
    else if (ty == 16) step_d2q9<COLL, ST, R, 16><<<g, b, 0, s>>>(d, bi, parity);
    else step_d2q9<COLL, ST, R, 12><<<g, b, 0, s>>>(d, bi, parity);
  } else {
    step_d3q19<COLL, ST, R><<<g, b, 0, s>>>(d, bi, parity);
  }
}

// Compacted 3D fused step of every instance (one launch over the block
// table), then per instance the pulled densities of its edge nodes and the
// virtual solid densities, into the carried psi of the next step.
template <int COLL, typename R>
static void launch_fwd_q(const StepLaunch &L, hipStream_t s) {
  if (L.n_blocks == 0) return;  // every instance retired
  fwd_step_d3q19<COLL, R><<<dim3((unsigned)L.n_blocks), dim3(kFwdThreads), 0, s>>>(L.d_insts, L.block_inst,
                                                                                  L.parity);
  for (int i = 0; i < L.k; ++i) {
    if (!L.live(i)) continue;
    const InstDev &h = L.h[i];
    if (h.nedge)
      fwd_rho_kernel<19><<<dim3((unsigned)((h.nedge + 255) / 256)), dim3(256), 0, s>>>(L.d_insts + i, h.cedge,
                                                                                      h.nedge, L.parity ^ 1);
    if (h.nbnd)
      fwd_ivsd_kernel<19><<<dim3((unsigned)((h.nbnd + 255) / 256)), dim3(256), 0, s>>>(L.d_insts + i, L.parity ^ 1);
  }
}

template <int COLL, int ST, typename R>
static void launch_fused_list_q(int q, int ty, const InstDev *d, const int32_t *bi, int64_t nb, int parity,
                                hipStream_t s) {
  const dim3 g((unsigned)nb), b(256);
  if (q != 9) return;
  if (ty == 8) step_d2q9_list<COLL, ST, R, 8><<<g, b, 0, s>>>(d, bi, parity);
  else if (ty == 16) step_d2q9_list<COLL, ST, R, 16><<<g, b, 0, s>>>(d, bi, parity);
  else step_d2q9_list<COLL, ST, R, 12><<<g, b, 0, s>>>(d, bi, parity);
}

template <int COLL, int ST, typename R>
static void launch_split_q(int q, const InstDev *d, const InstDev &h, int parity, hipStream_t s) {
  const int64_t waves = (int64_t)((h.nx + 63) / 64) * h.ny * h.nz;
  const dim3 g((unsigned)((waves + 3) / 4)), b(256);
  if (q == 9) {
    rho_kernel<9, ST><<<g, b, 0, s>>>(d, parity);
    psi_kernel<9><<<g, b, 0, s>>>(d);
    collide_kernel<9, COLL, ST, R><<<g, b, 0, s>>>(d, parity);
  } else {
    rho_kernel<19, ST><<<g, b, 0, s>>>(d, parity);
    psi_kernel<19><<<g, b, 0, s>>>(d);
    collide_kernel<19, COLL, ST, R><<<g, b, 0, s>>>(d, parity);
  }
}

template <int COLL, int ST, typename R>
static void launch_compact_q(int q, const InstDev *d, const InstDev &h, int parity, hipStream_t s) {
  if (h.nf == 0) return;  // no fluid: nothing moves
  const dim3 g((unsigned)((h.nf + kCompactThreads - 1) / kCompactThreads)), b(kCompactThreads);
  const dim3 gb((unsigned)((h.nbnd + 255) / 256)), bb(256);
  if (q == 9) {
    crho_kernel<9, ST><<<g, b, 0, s>>>(d, parity);
    if (h.nbnd) cpsi_kernel<9><<<gb, bb, 0, s>>>(d);
    ccollide_kernel<9, COLL, ST, R><<<g, b, 0, s>>>(d, parity);
  } else {
    crho_kernel<19, ST><<<g, b, 0, s>>>(d, parity);
    if (h.nbnd) cpsi_kernel<19><<<gb, bb, 0, s>>>(d);
    ccollide_kernel<19, COLL, ST, R><<<g, b, 0, s>>>(d, parity);
  }
}

// One step of every instance of a batch, for one collision operator: the
// storage, node arithmetic and strategy decide the kernels (see StepLaunch).
template <int COLL, int ST, typename R>
static void launch_st(const StepLaunch &L, hipStream_t s) {
  if (L.strategy == 2) {
    for (int i = 0; i < L.k; ++i)
      if (L.live(i)) launch_split_q<COLL, ST, R>(L.q, L.d_insts + i, L.h[i], L.parity, s);
  } else if (L.strategy == 3) {
    for (int i = 0; i < L.k; ++i)
      if (L.live(i)) launch_compact_q<COLL, ST, R>(L.q, L.d_insts + i, L.h[i], L.parity, s);
  } else if (L.n_blocks == 0) {
    return;  // block-table strategies with every instance retired: nothing to launch
  } else if (L.strategy == 4) {
    launch_fused_list_q<COLL, ST, R>(L.q, L.ty, L.d_insts, L.block_inst, L.n_blocks, L.parity, s);
  } else if (L.strategy == 5 && L.q == 19) {
    if constexpr (ST == 0) launch_fwd_q<COLL, R>(L, s);
  } else if (L.strategy == 5) {
    launch_fused_q<COLL, ST, R>(L.q, L.ty, L.d_insts, L.block_inst, L.n_blocks, L.parity, s, true);
  } else {
    launch_fused_q<COLL, ST, R>(L.q, L.ty, L.d_insts, L.block_inst, L.n_blocks, L.parity, s);
  }
}

template <int COLL>
hipError_t launch_step_coll(const StepLaunch &L, hipStream_t s) {
  if (L.math == LBM_MATH_F64) {
    if (L.storage == LBM_STORE_F32) launch_st<COLL, 0, double>(L, s);
    else launch_st<COLL, 1, double>(L, s);
  } else {
    if (L.storage == LBM_STORE_F32) launch_st<COLL, 0, float>(L, s);
    else launch_st<COLL, 1, float>(L, s);
  }
  return hipGetLastError();
}

}  // namespace lbm
