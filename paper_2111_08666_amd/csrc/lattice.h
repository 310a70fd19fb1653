// Lattice constants and node-local arithmetic of the two-component
// pseudopotential LBM (Sedahmed, Coelho & Warda, arXiv:2111.08666, Sec. 2),
// written for the GPU.  Everything here is inlined into the kernels.
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
  static constexpr double w[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                                  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

// D3Q19: rest, 6 axis links (w = 1/18), 12 face diagonals (w = 1/36); each
// odd index is followed by its opposite.
template <> struct Lat<19> {
  static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  static constexpr double w[19] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                   1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

// ---------------------------------------------------------------------------
// Node arithmetic runs in the type R (float by default, double optional);
// populations are held and stored as float, density sums run in double.
// ---------------------------------------------------------------------------

// Zou-He pressure completion at an x face (Eqs. 18-25): given the density
// rho_b and zero tangential velocity, the links pointing into the domain
// (e_x == dir) are rebuilt from their opposites, the normal mass flux
// m = rho_b - (sum of tangential links) - 2 (sum of outgoing links), and the
// tangential momentum of the face-parallel links.  D2Q9: Eqs. 19-21 / 23-25;
// D3Q19: the on-site rule of Hecht & Harting (2010).
template <int Q, typename R>
__device__ __forceinline__ void zou_he(float (&f)[Q], R rho_b, int dir) {
  using L = Lat<Q>;
  R par = 0, out = 0, ny_ = 0, nz_ = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (L::ex[i] == 0) {
      par += (R)f[i];
      if (L::ey[i]) ny_ += L::ey[i] * (R)f[i];
      if (L::ez[i]) nz_ += L::ez[i] * (R)f[i];
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
    if (L::ex[i] == -dir) out += (R)f[i];
  const R m = rho_b - par - R(2) * out;
  ny_ *= R(0.5);
  nz_ *= R(0.5);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (L::ex[i] == dir) {
      R v = (R)f[L::opp[i]] + R(6) * (R)L::w[i] * m;
      if (L::ey[i]) v -= L::ey[i] * ny_;
      if (L::ez[i]) v -= L::ez[i] * nz_;
      f[i] = (float)v;
    }
  }
}

// Inlet / outlet completion of one node for both components (Sec. 2.3).
// own(c, i) returns this node's post-collision value (Eq. 28),
// frozen(c, i) the held initial value (Eq. 26, Eq. 27; with eq26_mode 1
// those links take own(c, i) as well).
template <int Q, typename R, class OwnF, class FrozenF>
__device__ __forceinline__ void complete_boundary(const InstDev &d, uint32_t info, float (&f0)[Q],
                                                  float (&f1)[Q], OwnF own, FrozenF frozen) {
  using L = Lat<Q>;
  if (info & kInlet) {
    zou_he<Q, R>(f0, (R)d.rho_in1, +1);  // component 1: Eqs. 22-25
    if (d.bc_set == 1) {
      zou_he<Q, R>(f1, (R)d.rho_in2, +1);
    } else if (d.bc_set == 2) {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (L::ex[i] > 0) f1[i] = d.eq26_mode ? own(1, i) : frozen(1, i);  // Eq. 27
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (L::ex[i] > 0) f1[i] = own(1, i);  // Eq. 28
    }
  }
  if (info & kOutlet) {
    zou_he<Q, R>(f1, (R)d.rho_out2, -1);  // component 2: Eqs. 18-21
    if (d.bc_set == 1) {
      zou_he<Q, R>(f0, (R)d.rho_out1, -1);
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (L::ex[i] < 0) f0[i] = d.eq26_mode ? own(0, i) : frozen(0, i);  // Eq. 26
    }
  }
}

// Reciprocal: hardware estimate refined by two Newton steps (to full
// precision in double, correctly rounded in nearly every case in float).
template <typename R> __device__ __forceinline__ R rcp(R x);
template <> __device__ __forceinline__ double rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
template <> __device__ __forceinline__ float rcp<float>(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  float e = __builtin_fmaf(-x, r, 1.f);
  r = __builtin_fmaf(r, e, r);
  e = __builtin_fmaf(-x, r, 1.f);
  return __builtin_fmaf(r, e, r);
}

// Sum of the populations, pairing opposite links first; accumulated in FP64
// whatever the node arithmetic (the density is then rounded once).
template <int Q, typename R>
__device__ __forceinline__ R sum_q(const float (&f)[Q]) {
  double s = (double)f[0];
#pragma unroll
  for (int i = 1; i < Q; ++i)
    if (Lat<Q>::opp[i] > i) s += (double)f[i] + (double)f[Lat<Q>::opp[i]];
  return (R)s;
}

// D3Q19 moment basis of d'Humieres, Ginzburg, Krafczyk, Lallemand & Luo
// (2002): entry (k, i) of the moment matrix, rows rho, e, eps, jx, qx, jy,
// qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz.  The rows are
// mutually orthogonal, so the inverse is the transpose over the row norms.
__host__ __device__ constexpr int mrt19(int k, int i) {
  const int cx = Lat<19>::ex[i], cy = Lat<19>::ey[i], cz = Lat<19>::ez[i];
  const int c2 = cx * cx + cy * cy + cz * cz;
  switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return cx;
    case 4: return (5 * c2 - 9) * cx;
    case 5: return cy;
    case 6: return (5 * c2 - 9) * cy;
    case 7: return cz;
    case 8: return (5 * c2 - 9) * cz;
    case 9: return 3 * cx * cx - c2;
    case 10: return (3 * c2 - 5) * (3 * cx * cx - c2);
    case 11: return cy * cy - cz * cz;
    case 12: return (3 * c2 - 5) * (cy * cy - cz * cz);
    case 13: return cx * cy;
    case 14: return cy * cz;
    case 15: return cx * cz;
    case 16: return (cy * cy - cz * cz) * cx;
    case 17: return (cz * cz - cx * cx) * cy;
    default: return (cx * cx - cy * cy) * cz;
  }
}
__host__ __device__ constexpr int mrt19_norm(int k) {
  int n = 0;
  for (int i = 0; i < 19; ++i) n += mrt19(k, i) * mrt19(k, i);
  return n;
}

// ---------------------------------------------------------------------------
// Relaxation rates at a node.  tau_s is the density-weighted mean of the
// component relaxation times (Eq. 6 with nu = (tau - 1/2)/3); the shear rate
// is 1/tau_s, the odd (energy-flux) rate follows the magic parameter lambda.
// ---------------------------------------------------------------------------
template <typename R> struct Rates {
  R s_nu, s_q, s_e, s_eps, s_j;
};

template <typename R>
__device__ __forceinline__ Rates<R> node_rates(const InstDev &d, R rho1, R rho2, R inv_rho) {
  Rates<R> r;
  const R tau_s = (rho1 * (R)d.tau1 + rho2 * (R)d.tau2) * inv_rho;
  r.s_nu = rcp<R>(tau_s);
  // 1/s_q = 1/2 + lambda/(tau_s - 1/2)  =>  s_q = (tau_s - 1/2) / ((tau_s - 1/2)/2 + lambda)
  const R a = tau_s - R(0.5);
  r.s_q = d.lambda > 0 ? a * rcp<R>(R(0.5) * a + (R)d.lambda) : r.s_nu;
  r.s_e = d.s_e > 0 ? (R)d.s_e : r.s_nu;
  r.s_eps = d.s_eps > 0 ? (R)d.s_eps : r.s_nu;
  // component-momentum rate: 0 the smaller of s_nu and s_q, 1 s_q, 2 s_nu
  r.s_j = d.sj_mode == 1 ? r.s_q : (d.sj_mode == 2 ? r.s_nu : (r.s_nu < r.s_q ? r.s_nu : r.s_q));
  return r;
}

// Fused multiply-add in the node arithmetic's type (one rounding).
template <typename R> __device__ __forceinline__ R fmar(R a, R b, R c);
template <> __device__ __forceinline__ double fmar<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <> __device__ __forceinline__ float fmar<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Departure of population i from the equilibrium (Eq. 2) and its source
// term (Eq. 11) at velocity u with force F:
//   feq_i - f_i = (w_i rho - f_i) + w_i rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u),
// the first term formed in one rounding (fused multiply-add), so that a
// population near its rest equilibrium loses nothing to cancellation.
template <int Q, typename R>
__device__ __forceinline__ void departure(int i, float f, R rho, R ux, R uy, R uz, R Fx, R Fy, R Fz, R usq15,
                                          R uF, R &dv, R &S) {
  using L = Lat<Q>;
  const R eu = L::ex[i] * ux + L::ey[i] * uy + L::ez[i] * uz;
  const R eF = L::ex[i] * Fx + L::ey[i] * Fy + L::ez[i] * Fz;
  const R w = (R)L::w[i];
  dv = fmar<R>(w, rho, -(R)f) + w * rho * (R(3) * eu + R(4.5) * eu * eu - usq15);
  S = w * (R(3) * (eF - uF) + R(9) * eu * eF);
}

// ---------------------------------------------------------------------------
// Forced collision of one component at one node, in place (Eqs. 1, 2, 11).
// u: common velocity (with the half-force shift), F: this component's force.
// COLL: 0 SRT, 1 MRT (D2Q9: Lallemand-Luo moments; D3Q19: d'Humieres), 2 TRT.
// Each moving population changes by an increment built from its departure
// from equilibrium; the rest population takes minus their sum, so the node
// keeps its mass to the rounding of the stores.
// ---------------------------------------------------------------------------
template <int Q, int COLL, typename R>
__device__ __forceinline__ void collide_component(float (&fo)[Q], R rho, R ux, R uy, R uz, R Fx,
                                                  R Fy, R Fz, const Rates<R> &r) {
  using L = Lat<Q>;
  const R usq15 = R(1.5) * (ux * ux + uy * uy + uz * uz);
  const R uF = ux * Fx + uy * Fy + uz * Fz;
  R moved = 0;  // sum of the moving populations' changes
  if constexpr (COLL == 0) {
    const R om = r.s_nu, fac = R(1) - R(0.5) * om;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      R dv, S;
      departure<Q, R>(i, fo[i], rho, ux, uy, uz, Fx, Fy, Fz, usq15, uF, dv, S);
      const R df = om * dv + fac * S;
      fo[i] = (float)((R)fo[i] + df);
      moved += df;
    }
  } else if constexpr (COLL == 2) {
    const R sp = r.s_nu, sm = r.s_q;
    const R fp = R(1) - R(0.5) * sp, fm = R(1) - R(0.5) * sm;
    // opposite pairs (i, b): the pair's symmetric and antisymmetric parts
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int b = L::opp[i];
      if (b < i) continue;
      // e_b = -e_i: the pair shares e.u and e.F up to sign, so the
      // departures' halves come from one evaluation of each
      const R eu = L::ex[i] * ux + L::ey[i] * uy + L::ez[i] * uz;
      const R eF = L::ex[i] * Fx + L::ey[i] * Fy + L::ez[i] * Fz;
      const R w = (R)L::w[i], wr = w * rho;
      const R ai = fmar<R>(w, rho, -(R)fo[i]), ab = fmar<R>(w, rho, -(R)fo[b]);
      const R dv_p = R(0.5) * (ai + ab) + wr * (R(4.5) * eu * eu - usq15);  // (dv_i + dv_b) / 2
      const R dv_m = R(0.5) * (ai - ab) + wr * R(3) * eu;                    // (dv_i - dv_b) / 2
      const R S_p = w * (R(9) * eu * eF - R(3) * uF), S_m = w * R(3) * eF;
      const R dp = sp * dv_p + fp * S_p;  // change of the symmetric part
      const R dm = sm * dv_m + fm * S_m;  // change of the antisymmetric part
      fo[i] = (float)((R)fo[i] + (dp + dm));
      fo[b] = (float)((R)fo[b] + (dp - dm));
      moved += R(2) * dp;
    }
  } else if constexpr (Q == 19) {
    // MRT in the d'Humieres moments: the second-order moments relax at s_nu,
    // e and eps at the free energy rates, pi at s_eps, j at s_j, q and m at
    // s_q (equal even and odd rates give TRT, equal rates give SRT).
    R dv[Q], S[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) departure<Q, R>(i, fo[i], rho, ux, uy, uz, Fx, Fy, Fz, usq15, uF, dv[i], S[i]);
    auto rate = [&](int k) -> R {
      switch (k) {
        case 1: return r.s_e;
        case 2: case 10: case 12: return r.s_eps;
        case 3: case 5: case 7: return r.s_j;
        case 4: case 6: case 8: case 16: case 17: case 18: return r.s_q;
        default: return r.s_nu;
      }
    };
    R dm[Q];
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      R a = 0, b = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (mrt19(k, i) != 0) {
          a += R(mrt19(k, i)) * dv[i];
          b += R(mrt19(k, i)) * S[i];
        }
      }
      const R sk = rate(k);
      dm[k] = (sk * a + (R(1) - R(0.5) * sk) * b) * (R(1) / R(mrt19_norm(k)));
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      R v = 0;
#pragma unroll
      for (int k = 1; k < Q; ++k)
        if (mrt19(k, i) != 0) v += R(mrt19(k, i)) * dm[k];
      fo[i] = (float)((R)fo[i] + v);
      moved += v;
    }
  } else {
    // D2Q9 MRT: moments (Lallemand-Luo rows e, eps, jx, qx, jy, qy, pxx,
    // pxy) of the departures from equilibrium and of the source
    R d[Q], S[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) departure<Q, R>(i, fo[i], rho, ux, uy, uz, Fx, Fy, Fz, usq15, uF, d[i], S[i]);
    auto mom = [](const R(&f)[Q], R(&m)[8]) {
      const R a = f[1] + f[2] + f[3] + f[4];
      const R dg = f[5] + f[6] + f[7] + f[8];
      const R d13 = f[1] - f[3], d24 = f[2] - f[4];
      const R p5 = f[5] - f[7], p6 = f[6] - f[8];
      m[0] = R(-4) * f[0] - a + R(2) * dg;      // e
      m[1] = R(4) * f[0] - R(2) * a + dg;       // eps
      m[2] = d13 + p5 - p6;                     // jx
      m[3] = R(-2) * d13 + p5 - p6;             // qx
      m[4] = d24 + p5 + p6;                     // jy
      m[5] = R(-2) * d24 + p5 + p6;             // qy
      m[6] = (f[1] + f[3]) - (f[2] + f[4]);     // pxx
      m[7] = (f[5] + f[7]) - (f[6] + f[8]);     // pxy
    };
    R md[8], ms[8];
    mom(d, md);
    mom(S, ms);
    const R sr[8] = {r.s_e, r.s_eps, r.s_j, r.s_q, r.s_j, r.s_q, r.s_nu, r.s_nu};
    R dmv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) dmv[k] = sr[k] * md[k] + (R(1) - R(0.5) * sr[k]) * ms[k];
    // f += M^-1 dm, M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    const R ce = dmv[0] * R(1.0 / 36.0), cp = dmv[1] * R(1.0 / 36.0);
    const R jx = dmv[2] * R(1.0 / 6.0), qx = dmv[3] * R(1.0 / 12.0);
    const R jy = dmv[4] * R(1.0 / 6.0), qy = dmv[5] * R(1.0 / 12.0);
    const R pxx = dmv[6] * R(0.25), pxy = dmv[7] * R(0.25);
    const R ax = -ce - R(2) * cp;
    const R dd = R(2) * ce + cp;
    const R df[Q] = {0,
                     ax + jx - R(2) * qx + pxx,
                     ax + jy - R(2) * qy - pxx,
                     ax - jx + R(2) * qx + pxx,
                     ax - jy + R(2) * qy - pxx,
                     dd + jx + qx + jy + qy + pxy,
                     dd - jx - qx + jy + qy - pxy,
                     dd - jx - qx - jy - qy + pxy,
                     dd + jx + qx - jy - qy - pxy};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      fo[i] = (float)((R)fo[i] + df[i]);
      moved += df[i];
    }
  }
  fo[0] = (float)((R)fo[0] - moved);
}

// Mixture velocity, rates and the collision of both components at a node.
// rho1/rho2 are the node densities, F the per-component forces
// (interaction + body).
template <int Q, int COLL, typename R>
__device__ __forceinline__ void collide_node(const InstDev &d, float (&f0)[Q], float (&f1)[Q], R rho1,
                                             R rho2, R F1x, R F1y, R F1z, R F2x, R F2y, R F2z) {
  using L = Lat<Q>;
  // momentum summed over opposite pairs
  R jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (L::opp[i] < i) continue;
    const R dsum = ((R)f0[i] - (R)f0[L::opp[i]]) + ((R)f1[i] - (R)f1[L::opp[i]]);
    if (L::ex[i]) jx += L::ex[i] * dsum;
    if (L::ey[i]) jy += L::ey[i] * dsum;
    if (L::ez[i]) jz += L::ez[i] * dsum;
  }
  // the FP64 copies made for the momentum are not kept for the collision
#pragma unroll
  for (int i = 0; i < Q; ++i) asm volatile("" : "+v"(f0[i]), "+v"(f1[i]));
  const R rho = rho1 + rho2, inv_rho = rcp<R>(rho);
  const R h = d.half_shift ? R(0.5) : R(0);
  const R ux = (jx + h * (F1x + F2x)) * inv_rho;
  const R uy = (jy + h * (F1y + F2y)) * inv_rho;
  const R uz = (jz + h * (F1z + F2z)) * inv_rho;
  const Rates<R> r = node_rates<R>(d, rho1, rho2, inv_rho);
  collide_component<Q, COLL, R>(f0, rho1, ux, uy, uz, F1x, F1y, F1z, r);
  collide_component<Q, COLL, R>(f1, rho2, ux, uy, uz, F2x, F2y, F2z, r);
}

// ---------------------------------------------------------------------------
// BF16 deviation storage: per component and node the density rho (FP32) and
// d_i = f*_i - w_i rho for i >= 1 (BF16, round to nearest even).  The rest
// population is implicit, f*_0 = rho - sum_i f*_i, so the stored state
// holds each node's mass exactly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

}  // namespace lbm
