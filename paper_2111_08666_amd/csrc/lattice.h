// Lattice constants and node-local arithmetic of the two-component
// pseudopotential LBM (Sedahmed, Coelho & Warda, arXiv:2111.08666, Sec. 2),
// written for the GPU in FP32.  Everything here is inlined into the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"

namespace lbm {

template <int Q> struct Lat;

// D2Q9 in the paper's order (Sec. 2.1): rest, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-).
template <> struct Lat<9> {
  static constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  static constexpr float w[9] = {4.f / 9.f,  1.f / 9.f,  1.f / 9.f,  1.f / 9.f, 1.f / 9.f,
                                 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
};

// D3Q19: rest, 6 axis links (w = 1/18), 12 face diagonals (w = 1/36); each
// odd index is followed by its opposite.
template <> struct Lat<19> {
  static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  static constexpr float w[19] = {1.f / 3.f,  1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f,
                                  1.f / 18.f, 1.f / 18.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                  1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                  1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
};

// ---------------------------------------------------------------------------
// Zou-He pressure completion at an x face (Eqs. 18-25): given the density
// rho_b and zero tangential velocity, the links pointing into the domain
// (e_x == dir) are rebuilt from their opposites, the normal mass flux
// m = rho_b - (sum of tangential links) - 2 (sum of outgoing links), and the
// tangential momentum of the face-parallel links.  D2Q9: Eqs. 19-21 / 23-25;
// D3Q19: the on-site rule of Hecht & Harting (2010).
// ---------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ void zou_he(float (&f)[Q], float rho_b, int dir) {
  using L = Lat<Q>;
  float par = 0.f, out = 0.f, ny_ = 0.f, nz_ = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (L::ex[i] == 0) {
      par += f[i];
      if (L::ey[i]) ny_ += L::ey[i] * f[i];
      if (L::ez[i]) nz_ += L::ez[i] * f[i];
    }
  }
  if (dir > 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (L::ex[i] < 0) out += f[i];
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (L::ex[i] > 0) out += f[i];
  }
  const float m = rho_b - par - 2.f * out;
  ny_ *= 0.5f;
  nz_ *= 0.5f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (L::ex[i] == dir) {
      float v = f[L::opp[i]] + 6.f * L::w[i] * m;
      if (L::ey[i]) v -= L::ey[i] * ny_;
      if (L::ez[i]) v -= L::ez[i] * nz_;
      f[i] = v;
    }
  }
}

// Inlet / outlet completion of one node for both components (Sec. 2.3).
// own(c, i) returns this node's post-collision value (Eq. 28),
// frozen(c, i) the held initial value (Eq. 26, Eq. 27).
template <int Q, class OwnF, class FrozenF>
__device__ __forceinline__ void complete_boundary(const InstDev &d, uint32_t info, float (&f0)[Q],
                                                  float (&f1)[Q], OwnF own, FrozenF frozen) {
  using L = Lat<Q>;
  if (info & kInlet) {
    zou_he<Q>(f0, d.rho_in1, +1);  // component 1: Eqs. 22-25
    if (d.bc_set == 1) {
      zou_he<Q>(f1, d.rho_in2, +1);
    } else if (d.bc_set == 2) {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (L::ex[i] > 0) f1[i] = frozen(1, i);  // Eq. 27
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (L::ex[i] > 0) f1[i] = own(1, i);  // Eq. 28
    }
  }
  if (info & kOutlet) {
    zou_he<Q>(f1, d.rho_out2, -1);  // component 2: Eqs. 18-21
    if (d.bc_set == 1) {
      zou_he<Q>(f0, d.rho_out1, -1);
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (L::ex[i] < 0) f0[i] = frozen(0, i);  // Eq. 26
    }
  }
}

// ---------------------------------------------------------------------------
// Relaxation rates at a node.  tau_s is the density-weighted mean of the
// component relaxation times (Eq. 6 with nu = (tau - 1/2)/3); the shear rate
// is 1/tau_s, the odd (energy-flux) rate follows the magic parameter lambda.
// ---------------------------------------------------------------------------
struct Rates {
  float s_nu, s_q, s_e, s_eps, s_j;
};

__device__ __forceinline__ Rates node_rates(const InstDev &d, float rho1, float rho2, float inv_rho) {
  Rates r;
  const float tau_s = (rho1 * d.tau1 + rho2 * d.tau2) * inv_rho;
  r.s_nu = 1.f / tau_s;
  r.s_q = d.lambda > 0.f ? 1.f / (0.5f + d.lambda / (tau_s - 0.5f)) : r.s_nu;
  r.s_e = d.s_e > 0.f ? d.s_e : r.s_nu;
  r.s_eps = d.s_eps > 0.f ? d.s_eps : r.s_nu;
  r.s_j = d.sj_mode ? r.s_q : r.s_nu;
  return r;
}

// ---------------------------------------------------------------------------
// Forced collision of one component at one node, in place (Eqs. 1, 2, 11).
// u: common velocity (with the half-force shift), F: this component's force.
// COLL: 0 SRT, 1 MRT (D2Q9 Lallemand-Luo moments), 2 TRT.
// ---------------------------------------------------------------------------
template <int Q, int COLL>
__device__ __forceinline__ void collide_component(float (&f)[Q], float rho, float ux, float uy,
                                                  float uz, float Fx, float Fy, float Fz,
                                                  const Rates &r) {
  using L = Lat<Q>;
  const float usq15 = 1.5f * (ux * ux + uy * uy + uz * uz);
  const float uF = ux * Fx + uy * Fy + uz * Fz;
  if constexpr (COLL == 0) {
    const float om = r.s_nu, fo = 1.f - 0.5f * om;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float eu = L::ex[i] * ux + L::ey[i] * uy + L::ez[i] * uz;
      const float eF = L::ex[i] * Fx + L::ey[i] * Fy + L::ez[i] * Fz;
      const float feq = L::w[i] * rho * (1.f + 3.f * eu + 4.5f * eu * eu - usq15);
      const float S = L::w[i] * (3.f * (eF - uF) + 9.f * eu * eF);
      f[i] = f[i] + om * (feq - f[i]) + fo * S;
    }
  } else if constexpr (COLL == 2) {
    const float sp = r.s_nu, sm = r.s_q;
    const float fp = 1.f - 0.5f * sp, fm = 1.f - 0.5f * sm;
    float o[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int b = L::opp[i];
      const float eu = L::ex[i] * ux + L::ey[i] * uy + L::ez[i] * uz;
      const float eF = L::ex[i] * Fx + L::ey[i] * Fy + L::ez[i] * Fz;
      // symmetric / antisymmetric parts of feq and S
      const float eq_p = L::w[i] * rho * (1.f + 4.5f * eu * eu - usq15);
      const float eq_m = L::w[i] * rho * 3.f * eu;
      const float S_p = L::w[i] * (9.f * eu * eF - 3.f * uF);
      const float S_m = L::w[i] * 3.f * eF;
      const float f_p = 0.5f * (f[i] + f[b]), f_m = 0.5f * (f[i] - f[b]);
      o[i] = f[i] + sp * (eq_p - f_p) + sm * (eq_m - f_m) + fp * S_p + fm * S_m;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = o[i];
  } else {
    static_assert(Q == 9, "MRT is D2Q9 only");
    // moments of the deviation from the rest state: only non-conserved rows
    const float a = f[1] + f[2] + f[3] + f[4];
    const float dg = f[5] + f[6] + f[7] + f[8];
    const float m_e = -4.f * f[0] - a + 2.f * dg;
    const float m_eps = 4.f * f[0] - 2.f * a + dg;
    const float d13 = f[1] - f[3], d24 = f[2] - f[4];
    const float p5 = f[5] - f[7], p6 = f[6] - f[8];
    const float m_jx = d13 + p5 - p6;
    const float m_qx = -2.f * d13 + p5 - p6;
    const float m_jy = d24 + p5 + p6;
    const float m_qy = -2.f * d24 + p5 + p6;
    const float m_pxx = (f[1] + f[3]) - (f[2] + f[4]);
    const float m_pxy = (f[5] + f[7]) - (f[6] + f[8]);
    const float u2 = ux * ux + uy * uy;
    // equilibrium moments of Eq. 2 and moments of the source of Eq. 11
    const float e_eq = rho * (-2.f + 3.f * u2), eps_eq = rho * (1.f - 3.f * u2);
    const float jx_eq = rho * ux, jy_eq = rho * uy;
    const float pxx_eq = rho * (ux * ux - uy * uy), pxy_eq = rho * ux * uy;
    const float S_e = 6.f * uF, S_eps = -6.f * uF;
    const float S_pxx = 2.f * (ux * Fx - uy * Fy), S_pxy = ux * Fy + uy * Fx;
    const float dm_e = r.s_e * (e_eq - m_e) + (1.f - 0.5f * r.s_e) * S_e;
    const float dm_eps = r.s_eps * (eps_eq - m_eps) + (1.f - 0.5f * r.s_eps) * S_eps;
    const float dm_jx = r.s_j * (jx_eq - m_jx) + (1.f - 0.5f * r.s_j) * Fx;
    const float dm_jy = r.s_j * (jy_eq - m_jy) + (1.f - 0.5f * r.s_j) * Fy;
    const float dm_qx = r.s_q * (-jx_eq - m_qx) - (1.f - 0.5f * r.s_q) * Fx;
    const float dm_qy = r.s_q * (-jy_eq - m_qy) - (1.f - 0.5f * r.s_q) * Fy;
    const float dm_pxx = r.s_nu * (pxx_eq - m_pxx) + (1.f - 0.5f * r.s_nu) * S_pxx;
    const float dm_pxy = r.s_nu * (pxy_eq - m_pxy) + (1.f - 0.5f * r.s_nu) * S_pxy;
    // f += M^-1 dm, M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    const float ce = dm_e * (1.f / 36.f), cp = dm_eps * (1.f / 36.f);
    const float jx = dm_jx * (1.f / 6.f), qx = dm_qx * (1.f / 12.f);
    const float jy = dm_jy * (1.f / 6.f), qy = dm_qy * (1.f / 12.f);
    const float pxx = dm_pxx * 0.25f, pxy = dm_pxy * 0.25f;
    f[0] += -4.f * ce + 4.f * cp;
    const float ax = -ce - 2.f * cp;
    f[1] += ax + jx - 2.f * qx + pxx;
    f[2] += ax + jy - 2.f * qy - pxx;
    f[3] += ax - jx + 2.f * qx + pxx;
    f[4] += ax - jy + 2.f * qy - pxx;
    const float dd = 2.f * ce + cp;
    f[5] += dd + jx + qx + jy + qy + pxy;
    f[6] += dd - jx - qx + jy + qy - pxy;
    f[7] += dd - jx - qx - jy - qy + pxy;
    f[8] += dd + jx + qx - jy - qy - pxy;
  }
}

// Mixture velocity, rates and the collision of both components at a node.
// rho1/rho2 are the node densities (sums of f0/f1), F the per-component
// forces (interaction + body).
template <int Q, int COLL>
__device__ __forceinline__ void collide_node(const InstDev &d, float (&f0)[Q], float (&f1)[Q],
                                             float rho1, float rho2, float F1x, float F1y,
                                             float F1z, float F2x, float F2y, float F2z) {
  using L = Lat<Q>;
  // momentum summed over opposite pairs: differences of nearby values
  float jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (L::opp[i] < i) continue;
    const float d0 = f0[i] - f0[L::opp[i]], d1 = f1[i] - f1[L::opp[i]];
    const float dsum = d0 + d1;
    if (L::ex[i]) jx += L::ex[i] * dsum;
    if (L::ey[i]) jy += L::ey[i] * dsum;
    if (L::ez[i]) jz += L::ez[i] * dsum;
  }
  const float rho = rho1 + rho2, inv_rho = 1.f / rho;
  const float h = d.half_shift ? 0.5f : 0.f;
  const float ux = (jx + h * (F1x + F2x)) * inv_rho;
  const float uy = (jy + h * (F1y + F2y)) * inv_rho;
  const float uz = (jz + h * (F1z + F2z)) * inv_rho;
  const Rates r = node_rates(d, rho1, rho2, inv_rho);
  collide_component<Q, COLL>(f0, rho1, ux, uy, uz, F1x, F1y, F1z, r);
  collide_component<Q, COLL>(f1, rho2, ux, uy, uz, F2x, F2y, F2z, r);
}

// ---------------------------------------------------------------------------
// BF16 deviation storage: per component and node the density rho (FP32) and
// d_i = f*_i - w_i rho for i >= 1 (BF16, round to nearest even).  The rest
// population is implicit, f*_0 = w_0 rho - sum_i d_i, so the stored state
// holds each node's mass exactly.
// Buffer layout: [rho planes: 2 x plane floats][d planes: 2 x (Q-1) x plane bf16]
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

}  // namespace lbm
