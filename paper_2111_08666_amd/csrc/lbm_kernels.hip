// HIP kernels for gfx950: the fused two-component step (D2Q9 and D3Q19),
// initialisation, observables and density extraction.
//
// State between steps: the post-collision populations f*^s_i(x) in a
// structure-of-arrays layout, plane (s, i) holding one value per node with x
// fastest (row pitch a multiple of 64 elements), two buffers in ping-pong.
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
typedef __attribute__((address_space(1))) uint16_t gu16;
typedef __attribute__((address_space(1))) const uint16_t gcu16;

__device__ __forceinline__ gcf *G(const float *p) { return (gcf *)p; }
__device__ __forceinline__ gf *G(float *p) { return (gf *)p; }

// ---------------------------------------------------------------------------
// population access by storage kind
// FP32:  buffer = [s][i][plane] floats
// BF16:  buffer = [s][plane] float densities, then [s][i-1][plane] bf16
//        deviations d_i = f*_i - w_i rho (i >= 1); f*_0 = w_0 rho - sum d_i.
// ---------------------------------------------------------------------------
template <int Q, int ST>
__device__ __forceinline__ float pop_get(gcf *__restrict__ b, int64_t plane, int s, int i, int64_t off) {
  if constexpr (ST == 0) {
    return b[(int64_t)(s * Q + i) * plane + off];
  } else {
    const float r = b[(int64_t)s * plane + off];
    gcu16 *dv = (gcu16 *)(b + 2 * plane);
    if (i == 0) {
      float sum = 0.f;
#pragma unroll
      for (int j = 1; j < Q; ++j) sum += bf16_to_f32(dv[(int64_t)(s * (Q - 1) + j - 1) * plane + off]);
      return (float)Lat<Q>::w[0] * r - sum;
    }
    return (float)Lat<Q>::w[i] * r + bf16_to_f32(dv[(int64_t)(s * (Q - 1) + i - 1) * plane + off]);
  }
}

// Store both components' post-collision populations of one node.
template <int Q, int ST>
__device__ __forceinline__ void pop_store(gf *__restrict__ b, int64_t plane, int64_t off,
                                          const float (&f0)[Q], const float (&f1)[Q], float rho1,
                                          float rho2) {
  if constexpr (ST == 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      b[(int64_t)i * plane + off] = f0[i];
      b[(int64_t)(Q + i) * plane + off] = f1[i];
    }
  } else {
    // collision conserves each component's node mass, so rho is stored as is
    b[off] = rho1;
    b[plane + off] = rho2;
    gu16 *dv = (gu16 *)(b + 2 * plane);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const float w = (float)Lat<Q>::w[i];
      dv[(int64_t)(i - 1) * plane + off] = f32_to_bf16(f0[i] - w * rho1);
      dv[(int64_t)(Q - 1 + i - 1) * plane + off] = f32_to_bf16(f1[i] - w * rho2);
    }
  }
}

// Inlet/outlet completion of one pulled node (links already pulled).
template <int Q, int ST, typename R>
__device__ __forceinline__ void complete(const InstDev &d, gcf *__restrict__ fin, uint32_t info, int y,
                                         int z, int64_t off, float (&f0)[Q], float (&f1)[Q]) {
  const int t = y + d.ny * z;
  const int64_t nt = (int64_t)d.ny * d.nz;
  gcf *frz = G(d.frozen);
  complete_boundary<Q, R>(
      d, info, f0, f1, [&](int s, int i) { return pop_get<Q, ST>(fin, d.plane, s, i, off); },
      [&](int s, int i) { return frz[(int64_t)(s * Q + i) * nt + t]; });
}

// ---------------------------------------------------------------------------
// Pull one fluid node's populations for both components: f_i(x) = f*_i(x-e_i),
// or this node's f*_opp(i) where x - e_i is solid.  Every address is valid:
// sources wrap periodically, and a wrapped source across an open face is a
// missing link whose value complete() overwrites.
// ---------------------------------------------------------------------------
template <int Q, int ST>
__device__ __forceinline__ void pull(const InstDev &d, gcf *__restrict__ fin, uint32_t info, int x, int y,
                                     int z, float (&f0)[Q], float (&f1)[Q]) {
  using L = Lat<Q>;
  const int64_t plane = d.plane;
  const int64_t rowp = d.pitch;
  const int64_t slab = (int64_t)d.pitch * d.ny;
  const int64_t off = x + rowp * y + slab * z;
  const int xm = x == 0 ? d.nx - 1 : x - 1, xp = x == d.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? d.ny - 1 : y - 1, yp = y == d.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? d.nz - 1 : z - 1, zp = z == d.nz - 1 ? 0 : z + 1;
  const int64_t xs[3] = {xp, x, xm};  // source x for e_x = -1, 0, +1
  const int64_t ys[3] = {yp * rowp, y * rowp, ym * rowp};
  const int64_t zs[3] = {zp * slab, z * slab, zm * slab};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const bool bb = (info >> i) & 1u;
    const int64_t src = xs[L::ex[i] + 1] + ys[L::ey[i] + 1] + zs[L::ez[i] + 1];
    const int64_t o = bb ? off : src;
    const int pi = bb ? L::opp[i] : i;
    if constexpr (ST == 0) {
      f0[i] = fin[(int64_t)pi * plane + o];
      f1[i] = fin[(int64_t)(Q + pi) * plane + o];
    } else {
      f0[i] = pop_get<Q, 1>(fin, plane, 0, pi, o);
      f1[i] = pop_get<Q, 1>(fin, plane, 1, pi, o);
    }
  }
}

// pull + inlet/outlet completion.  (x, y, z) are in-domain coordinates.
template <int Q, int ST, typename R>
__device__ __forceinline__ void gather(const InstDev &d, gcf *__restrict__ fin, uint32_t info,
                                       int x, int y, int z, float (&f0)[Q], float (&f1)[Q]) {
  pull<Q, ST>(d, fin, info, x, y, z, f0, f1);
  if (info & (kInlet | kOutlet))
    complete<Q, ST, R>(d, fin, info, y, z, x + (int64_t)d.pitch * (y + (int64_t)d.ny * z), f0, f1);
}

// Blocks are dealt round-robin to the 8 XCDs; renumber them so each XCD
// works on a contiguous range of tiles and neighbouring tiles share its L2.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7;
  return xcd * q8 + min(xcd, r8) + (b >> 3);
}

// ---------------------------------------------------------------------------
// D2Q9 fused step.  Block = 4 waves over a region of 64 columns x 16 rows:
// 60 x 12 interior nodes plus a 2-node halo.  Wave w owns interior rows
// 2 + w + 4k (k = 0..2) and one halo row.
// Phase 1: pull + complete + densities for all 64 x 16 region nodes -> LDS.
// Phase 2: virtual solid density (Eq. 17) in place at solid region nodes.
// Phase 3: force (Eq. 13 with the open-face mirror) and collision for the
//          interior nodes, whose pulled populations stayed in registers.
// ---------------------------------------------------------------------------
constexpr int kRH = kTileY + 4;

template <int COLL, int ST, typename R>
__global__ __launch_bounds__(256) void step_d2q9(const InstDev *__restrict__ insts,
                                                  const int32_t *__restrict__ block_inst, int parity) {
  using L = Lat<9>;
  using V = Vec2<R>;
  __shared__ V psi[kRH][64];

  const int bid = xcd_block();
  const int inst = block_inst ? block_inst[bid] : 0;
  const InstDev &d = insts[inst];
  const int lb = bid - d.block_base;
  const int tx = lb % d.tiles_x, ty = lb / d.tiles_x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
    if (px) gx += gx < 0 ? nx : -nx;
    else col_in = false;
  }

  // rows owned: k = 0..2 interior (2 + wave + 4k), k = 3 halo
  int rows[4], gy[4];
  bool valid[4];
  uint32_t info[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    rows[k] = k < 3 ? 2 + wave + 4 * k : (wave < 2 ? wave : 12 + wave);
    int y = ty * kTileY - 2 + rows[k];
    bool in = col_in;
    if (y < 0 || y >= ny) {
      if (py) y += y < 0 ? ny : -ny;
      else in = false;
    }
    gy[k] = in ? y : 0;
    valid[k] = in;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) info[k] = valid[k] ? infop[gx + (int64_t)d.pitch * gy[k]] : kSolid;

  // Phase 1: issue every pull of this thread unconditionally (solid and
  // out-of-domain lanes read valid addresses inside the same cache lines and
  // discard the values), then complete and sum
  const int gxa = col_in ? gx : (gx < 0 ? 0 : nx - 1);
  float f0[3][9], f1[3][9], h0[9], h1[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) pull<9, ST>(d, fin, info[k], gxa, gy[k], 0, f0[k], f1[k]);
  pull<9, ST>(d, fin, info[3], gxa, gy[3], 0, h0, h1);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    R rho1 = 0, rho2 = 0;
    if (!(info[k] & kSolid)) {
      float(&a)[9] = k < 3 ? f0[k < 3 ? k : 0] : h0;
      float(&b)[9] = k < 3 ? f1[k < 3 ? k : 0] : h1;
      if (info[k] & (kInlet | kOutlet))
        complete<9, ST, R>(d, fin, info[k], gy[k], 0, gx + (int64_t)d.pitch * gy[k], a, b);
      rho1 = sum_q<9, R>(a);
      rho2 = sum_q<9, R>(b);
    }
    psi[rows[k]][lane] = V{rho1, rho2};
  }
  __syncthreads();

  // Phase 2: psi at solid nodes = chi^s * weighted mean of fluid-neighbour rho^s
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = rows[k];
    if (!valid[k] || !(info[k] & kSolid) || r < 1 || r > kRH - 2 || lane < 1 || lane > 62) continue;
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
  for (int k = 0; k < 3; ++k) {
    const int r = rows[k];
    const int gy_raw = ty * kTileY - 2 + r;
    if (!valid[k] || !col_store || gy_raw >= ny || (info[k] & kSolid)) continue;
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
    collide_node<9, COLL, R>(d, f0[k], f1[k], rho1, rho2, F1x, F1y, R(0), F2x, F2y, R(0));
    const int64_t off = gx + (int64_t)d.pitch * gy_raw;
    pop_store<9, ST>(fout, d.plane, off, f0[k], f1[k], (float)rho1, (float)rho2);
  }
}

// ---------------------------------------------------------------------------
// D3Q19 fused step.  A block owns a 60 x kTileY3 column of (x, y) and marches
// through z.  Per z plane it keeps densities of a 64 x (kTileY3 + 4) region in
// an LDS ring of five planes (z-2 .. z+2), completes psi at solid nodes of
// plane z+1 in place, and collides plane z with populations pulled two
// iterations earlier and held in registers.
// ---------------------------------------------------------------------------
constexpr int kRH3 = kTileY3 + 4;   // 8 region rows: wave w owns interior row 2+w and one halo row
constexpr int kRing = 5;

__device__ __forceinline__ int ring(int z) { return ((z % kRing) + kRing) % kRing; }

template <int COLL, int ST, typename R>
__global__ __launch_bounds__(256) void step_d3q19(const InstDev *__restrict__ insts,
                                                   const int32_t *__restrict__ block_inst, int parity) {
  using L = Lat<19>;
  using V = Vec2<R>;
  __shared__ V psi[kRing][kRH3][64];

  const int bid = xcd_block();
  const int inst = block_inst ? block_inst[bid] : 0;
  const InstDev &d = insts[inst];
  const int lb = bid - d.block_base;
  const int tx = lb % d.tiles_x, ty = (lb / d.tiles_x) % d.tiles_y;
  const int zc = lb / (d.tiles_x * d.tiles_y);  // z chunk
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  gcf *__restrict__ fin = G(d.f[parity]);
  gf *__restrict__ fout = G(d.f[parity ^ 1]);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const bool px = d.periodic & 1, py = d.periodic & 2, pz = d.periodic & 4;
  const int zlen = (nz + d.tiles_z - 1) / d.tiles_z;
  const int z0 = zc * zlen, z1 = min(nz, z0 + zlen);
  const int64_t slab = (int64_t)d.pitch * ny;

  int gx = tx * kTileX - 2 + lane;
  const bool col_store = lane >= 2 && lane < 62 && gx < nx;
  bool col_in = true;
  if (gx < 0 || gx >= nx) {
    if (px) gx += gx < 0 ? nx : -nx;
    else col_in = false;
  }
  // rows of this wave: interior row ri = 2 + wave, halo row rh
  const int ri = 2 + wave, rh = wave < 2 ? wave : 4 + wave;
  int gyi = ty * kTileY3 - 2 + ri, gyh = ty * kTileY3 - 2 + rh;
  const int gyi_raw = gyi;
  bool in_i = col_in, in_h = col_in;
  if (gyi < 0 || gyi >= ny) { if (py) gyi += gyi < 0 ? ny : -ny; else in_i = false; }
  if (gyh < 0 || gyh >= ny) { if (py) gyh += gyh < 0 ? ny : -ny; else in_h = false; }
  const bool store_ok = col_store && gyi_raw < ny;

  // plane index with periodic wrap; false if outside a closed z edge
  auto wrap_z = [&](int zp, int &zz) -> bool {
    zz = zp;
    if (zz < 0 || zz >= nz) {
      if (pz) { zz += zz < 0 ? nz : -nz; return true; }
      return false;
    }
    return true;
  };

  // densities of plane zp -> LDS ring; the interior node's pulled populations -> (a, b)
  auto load_plane = [&](int zp, float (&a)[19], float (&b)[19], uint32_t &inf_out) {
    const int slot = ring(zp);
    int zz;
    const bool zin = wrap_z(zp, zz);
    {
      R rho1 = 0, rho2 = 0;
      uint32_t inf = kSolid;
      if (in_i && zin) {
        inf = d.info[gx + (int64_t)d.pitch * gyi + slab * zz];
        if (!(inf & kSolid)) {
          gather<19, ST, R>(d, fin, inf, gx, gyi, zz, a, b);
          rho1 = sum_q<19, R>(a);
          rho2 = sum_q<19, R>(b);
        }
      }
      inf_out = inf;
      psi[slot][ri][lane] = V{rho1, rho2};
    }
    {
      R rho1 = 0, rho2 = 0;
      if (in_h && zin) {
        const uint32_t inf = d.info[gx + (int64_t)d.pitch * gyh + slab * zz];
        if (!(inf & kSolid)) {
          float ha[19], hb[19];
          gather<19, ST, R>(d, fin, inf, gx, gyh, zz, ha, hb);
          rho1 = sum_q<19, R>(ha);
          rho2 = sum_q<19, R>(hb);
        }
      }
      psi[slot][rh][lane] = V{rho1, rho2};
    }
  };

  // virtual solid density (Eq. 17) at the solid nodes of plane zp, in place;
  // reads rho at planes zp-1 .. zp+1
  auto solid_psi = [&](int zp) {
    const int slot = ring(zp);
    int zz;
    if (!wrap_z(zp, zz)) return;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = h ? rh : ri;
      const bool in = h ? in_h : in_i;
      if (!in || r < 1 || r > kRH3 - 2 || lane < 1 || lane > 62) continue;
      const uint32_t nb = d.info[gx + (int64_t)d.pitch * (h ? gyh : gyi) + slab * zz];
      if (!(nb & kSolid) || !(nb & kLinkMask)) continue;
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
      const R inv = R(1) / den;
      psi[slot][r][lane] = V{(R)d.chi1 * s1 * inv, (R)d.chi2 * s2 * inv};
    }
  };

  // force (Eq. 13 with the open-face mirror) + collision + store, plane z
  auto collide_plane = [&](int z, float (&a)[19], float (&b)[19], uint32_t inf) {
    if (!store_ok || (inf & kSolid)) return;
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
    const R G = (R)d.G, gxb = (R)d.gx, gyb = (R)d.gy, gzb = (R)d.gz;
    collide_node<19, COLL, R>(d, a, b, rho1, rho2, -G * rho1 * sx2 + rho1 * gxb,
                              -G * rho1 * sy2 + rho1 * gyb, -G * rho1 * sz2 + rho1 * gzb,
                              -G * rho2 * sx1 + rho2 * gxb, -G * rho2 * sy1 + rho2 * gyb,
                              -G * rho2 * sz1 + rho2 * gzb);
    const int64_t off = gx + (int64_t)d.pitch * gyi_raw + slab * z;
    pop_store<19, ST>(fout, d.plane, off, a, b, (float)rho1, (float)rho2);
  };

  // register ring: slot k holds the interior populations of plane z with (z - z0) % 3 == k
  float ra0[3][19], ra1[3][19];
  uint32_t rinf[3];
  // prologue: densities of planes z0-2 .. z0+1 (z0-2 and z0-1 only for the halo)
  load_plane(z0 - 2, ra0[1], ra1[1], rinf[1]);
  load_plane(z0 - 1, ra0[2], ra1[2], rinf[2]);
  load_plane(z0, ra0[0], ra1[0], rinf[0]);
  load_plane(z0 + 1, ra0[1], ra1[1], rinf[1]);
  __syncthreads();
  solid_psi(z0 - 1);
  solid_psi(z0);
  __syncthreads();

  auto body = [&](auto kc, int z) {
    constexpr int K = decltype(kc)::value;
    constexpr int K2 = (K + 2) % 3;
    load_plane(z + 2, ra0[K2], ra1[K2], rinf[K2]);
    __syncthreads();
    solid_psi(z + 1);  // needs rho at z .. z+2
    __syncthreads();
    collide_plane(z, ra0[K], ra1[K], rinf[K]);
    // ring slot of z-2 is rewritten at z+3: every read of it is behind this barrier
    __syncthreads();
  };
  for (int z = z0; z < z1; z += 3) {
    body(std::integral_constant<int, 0>{}, z);
    if (z + 1 < z1) body(std::integral_constant<int, 1>{}, z + 1);
    if (z + 2 < z1) body(std::integral_constant<int, 2>{}, z + 2);
  }
}

// ---------------------------------------------------------------------------
// initial state: f*_i = w_i rho0 at fluid nodes (rest equilibrium)
// ---------------------------------------------------------------------------
template <int Q, int ST>
__global__ void init_kernel(const InstDev *__restrict__ insts, const float *__restrict__ rho0, int parity) {
  const InstDev &d = insts[0];
  const int64_t n_nodes = (int64_t)d.nx * d.ny * d.nz;
  gf *b = G(d.f[parity]);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < n_nodes;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int x = n % d.nx;
    const int64_t yz = n / d.nx;
    const int64_t off = x + (int64_t)d.pitch * yz;
    const bool solid = d.info[off] & kSolid;
    const float r1 = solid ? 0.f : rho0[n], r2 = solid ? 0.f : rho0[n_nodes + n];
    float a[Q], c[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      a[i] = (float)(Lat<Q>::w[i] * (double)r1);
      c[i] = (float)(Lat<Q>::w[i] * (double)r2);
    }
    if constexpr (ST == 0) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        b[(int64_t)i * d.plane + off] = a[i];
        b[(int64_t)(Q + i) * d.plane + off] = c[i];
      }
    } else {
      pop_store<Q, 1>(b, d.plane, off, a, c, r1, r2);
    }
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
    gather<Q, ST, double>(d, fin, inf, x, y, z, a, b);
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

__global__ void obs_final(const double *__restrict__ partials, int n_blocks, double *__restrict__ out) {
  const int k = threadIdx.x;
  if (k >= kObsFields) return;
  double s = 0.0;
  int fl = 0;
  for (int b = 0; b < n_blocks; ++b) {
    const double v = partials[(int64_t)b * kObsFields + k];
    if (k == kObsFields - 1) fl |= (int)v;
    else s += v;
  }
  out[k] = (k == kObsFields - 1) ? (double)fl : s;
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
      gather<Q, ST, double>(d, fin, inf, x, y, z, a, b);
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

template <int COLL, int ST, typename R>
static void launch_step_q(int q, const InstDev *d, const int32_t *bi, int64_t nb, int parity,
                          hipStream_t s) {
  if (q == 9) step_d2q9<COLL, ST, R><<<dim3((unsigned)nb), dim3(256), 0, s>>>(d, bi, parity);
  else if constexpr (COLL != 1) step_d3q19<COLL, ST, R><<<dim3((unsigned)nb), dim3(256), 0, s>>>(d, bi, parity);
}

template <typename R>
static void launch_step_r(int q, int collision, int storage, const InstDev *d, const int32_t *bi,
                          int64_t nb, int parity, hipStream_t s) {
  if (storage == 0) {
    if (collision == 0) launch_step_q<0, 0, R>(q, d, bi, nb, parity, s);
    else if (collision == 1) launch_step_q<1, 0, R>(q, d, bi, nb, parity, s);
    else launch_step_q<2, 0, R>(q, d, bi, nb, parity, s);
  } else {
    if (collision == 0) launch_step_q<0, 1, R>(q, d, bi, nb, parity, s);
    else if (collision == 1) launch_step_q<1, 1, R>(q, d, bi, nb, parity, s);
    else launch_step_q<2, 1, R>(q, d, bi, nb, parity, s);
  }
}

hipError_t launch_step(const InstDev *d_insts, const int32_t *block_inst, int64_t n_blocks, int q,
                       int collision, int storage, int math, int parity, hipStream_t s) {
  if (math == 0) launch_step_r<double>(q, collision, storage, d_insts, block_inst, n_blocks, parity, s);
  else launch_step_r<float>(q, collision, storage, d_insts, block_inst, n_blocks, parity, s);
  return hipGetLastError();
}

const char *step_kernel_name(int q, int collision, int storage, int math) {
  static const char *lat[2] = {"step_d2q9", "step_d3q19"};
  static const char *coll[3] = {"SRT", "MRT", "TRT"};
  static const char *st[2] = {"f32", "bf16dev"};
  static const char *mt[2] = {"double", "float"};
  static thread_local char buf[96];
  snprintf(buf, sizeof buf, "%s<%s,%s,%s>", lat[q == 19], coll[collision], st[storage], mt[math]);
  return buf;
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
  obs_final<<<1, 64, 0, s>>>(partials, n_blocks, result);
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
