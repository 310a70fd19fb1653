// U-Net surrogate kernels for gfx950: implicit-GEMM convolutions on the BF16
// matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation), pooling,
// transposed convolution, the sigmoid head with a masked cross-entropy loss,
// and Adam.  C ABI in include/unet.h.
//
// MFMA operand layout (one wave, 32x32 output tile, K = 16 per instruction):
//   A fragment, lane l: A[row = l % 32][k = 8 * (l / 32) + j], j = 0..7
//   B fragment, lane l: B[k = 8 * (l / 32) + j][col = l % 32]
//   C, lane l, register r: C[row = 8 * (r / 4) + 4 * (l / 32) + r % 4][col = l % 32]
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>

#include "../../include/unet.h"

namespace unet {

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float floatx16 __attribute__((__vector_size__(16 * sizeof(float))));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f2bf(float v) {
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
  const uint4 v = *reinterpret_cast<const uint4 *>(p);
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }
__device__ __forceinline__ bf16x8 pack8(const uint16_t (&v)[8]) {
  uint4 u;
  u.x = v[0] | ((uint32_t)v[1] << 16);
  u.y = v[2] | ((uint32_t)v[3] << 16);
  u.z = v[4] | ((uint32_t)v[5] << 16);
  u.w = v[6] | ((uint32_t)v[7] << 16);
  return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ floatx16 mfma(bf16x8 a, bf16x8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int c_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// ---------------------------------------------------------------------------
// one MFMA, for checking the operand layout: C(32x32) = A(32x16) B(16x32),
// row-major, A/B BF16, C FP32
// ---------------------------------------------------------------------------
__global__ void mfma_probe_kernel(const uint16_t *A, const uint16_t *B, float *C) {
  const int l = threadIdx.x;
  uint16_t a[8], b[8];
  for (int j = 0; j < 8; ++j) {
    a[j] = A[(l % 32) * 16 + 8 * (l / 32) + j];
    b[j] = B[(8 * (l / 32) + j) * 32 + (l % 32)];
  }
  floatx16 acc = {};
  acc = mfma(pack8(a), pack8(b), acc);
  for (int r = 0; r < 16; ++r) C[c_row(r, l) * 32 + (l % 32)] = acc[r];
}

// ---------------------------------------------------------------------------
// Implicit-GEMM forward: C[p][co] = sum_k A(p, k) B(k, co).  Block = 4 waves,
// 64 x 64 output tile (2 x 2 waves of 32 x 32).
//   MODE 0, 3x3 convolution:  k = (tap, ci), A = x[p + off(tap)][ci] (zero
//          outside), B = w[co][tap][ci]; output at p.
//   MODE 1, transposed 2x2 convolution, tap = blockIdx.z: k = ci,
//          A = x[p][ci], B = w[co][tap][ci]; output at 2p + tap (grid 2h x 2w).
//   MODE 2, data gradient of the transposed convolution: k = (tap, co'),
//          A = dy[2p + tap][co'], B = wt[ci][tap][co'] (here the output
//          channel is ci, the reduction channel co').
// K chunks of 8 never straddle a tap because channel counts are multiples of 8.
// ---------------------------------------------------------------------------
struct GemmArgs {
  const uint16_t *x;  // A source
  int n, h, w;        // A-source grid for MODE 0/1 (= output grid for MODE 0); input grid for MODE 2
  int kc;             // reduction channels (cin for MODE 0/1, cout' for MODE 2)
  int x_cs, x_co;
  const uint16_t *wgt;
  const float *bias;
  int nout;           // output channels
  uint16_t *y;
  int y_cs, y_co;
  int relu;
};

// Wave tile TM x TN MFMA tiles (32 x 32 each): per K step a lane loads TM A
// fragments and TN B fragments for TM * TN products.  The four waves of a
// block are stacked along the pixels: block tile (128 TM) x (32 TN).
template <int MODE, int TM, int TN>
__global__ __launch_bounds__(256) void igemm_fwd(GemmArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t P = (int64_t)a.n * a.h * a.w;  // rows of A (pixels of the A grid)
  const int64_t pix0 = ((int64_t)blockIdx.x * 4 + wave) * (32 * TM);
  const int col0 = blockIdx.y * (32 * TN);
  const int tap_z = MODE == 1 ? (int)blockIdx.z : 0;
  const int half = lane >> 5;
  const int ntap = MODE == 0 ? 9 : (MODE == 2 ? 4 : 1);
  const int wtap = MODE == 1 ? 4 : ntap;  // taps per weight row
  const int K = ntap * a.kc;
  int pn[TM], py[TM], px[TM];
  bool prow[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const int64_t pix = pix0 + 32 * t + (lane & 31);
    prow[t] = pix < P;
    pn[t] = py[t] = px[t] = 0;
    if (prow[t]) {
      pn[t] = (int)(pix / ((int64_t)a.h * a.w));
      const int r = (int)(pix - (int64_t)pn[t] * a.h * a.w);
      py[t] = r / a.w;
      px[t] = r - py[t] * a.w;
    }
  }
  floatx16 acc[TM][TN];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[t][u] = floatx16{};
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int kk = k0 + 8 * half;
    bf16x8 A[TM], B[TN];
#pragma unroll
    for (int t = 0; t < TM; ++t) A[t] = zero8();
#pragma unroll
    for (int u = 0; u < TN; ++u) B[u] = zero8();
    if (kk < K) {
      const int tap = MODE == 1 ? tap_z : kk / a.kc;
      const int ch = kk - (MODE == 1 ? 0 : tap * a.kc);
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        if (!prow[t]) continue;
        if constexpr (MODE == 0) {
          const int yy = py[t] + tap / 3 - 1, xx = px[t] + tap % 3 - 1;
          if (yy >= 0 && yy < a.h && xx >= 0 && xx < a.w)
            A[t] = load8(a.x + ((int64_t)pn[t] * a.h * a.w + (int64_t)yy * a.w + xx) * a.x_cs + a.x_co + ch);
        } else if constexpr (MODE == 1) {
          const int64_t pix = pix0 + 32 * t + (lane & 31);
          A[t] = load8(a.x + pix * a.x_cs + a.x_co + ch);
        } else {
          const int H2 = 2 * a.h, W2 = 2 * a.w;
          const int yy = 2 * py[t] + (tap >> 1), xx = 2 * px[t] + (tap & 1);
          A[t] = load8(a.x + ((int64_t)pn[t] * H2 * W2 + (int64_t)yy * W2 + xx) * a.x_cs + a.x_co + ch);
        }
      }
#pragma unroll
      for (int u = 0; u < TN; ++u) {
        const int col = col0 + 32 * u + (lane & 31);
        if (col < a.nout) B[u] = load8(a.wgt + ((int64_t)col * wtap + tap) * a.kc + ch);
      }
    }
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
      for (int u = 0; u < TN; ++u) acc[t][u] = mfma(A[t], B[u], acc[t][u]);
  }
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int col = col0 + 32 * u + (lane & 31);
    if (col >= a.nout) continue;
    const float bv = a.bias ? a.bias[col] : 0.f;
#pragma unroll
    for (int t = 0; t < TM; ++t) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t p = pix0 + 32 * t + c_row(r, lane);
        if (p >= P) continue;
        float v = acc[t][u][r] + bv;
        if (a.relu) v = v > 0.f ? v : 0.f;
        int64_t o;
        if constexpr (MODE == 1) {
          const int qn = (int)(p / ((int64_t)a.h * a.w));
          const int rr = (int)(p - (int64_t)qn * a.h * a.w);
          const int qy = rr / a.w, qx = rr - qy * a.w;
          const int H2 = 2 * a.h, W2 = 2 * a.w;
          o = (int64_t)qn * H2 * W2 + (int64_t)(2 * qy + (tap_z >> 1)) * W2 + 2 * qx + (tap_z & 1);
        } else {
          o = p;
        }
        a.y[o * a.y_cs + a.y_co + col] = f2bf(v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 3x3 convolution with LDS staging.  The reduction runs over 16-channel
// groups, and within a group over the nine taps (k = (group, tap, channel)):
// per group the block stages its input rows with a one-pixel halo (zero
// outside the image) and the group's weights of its output channels in LDS
// once, and all nine taps of all four waves read their MFMA fragments from
// there.  Wave tile TM x TN MFMA tiles (32 x 32 each); the four waves are
// stacked along the pixels, so a block covers 128 TM consecutive pixels --
// whole image rows (16 <= w <= 256, w divides the block, h * w a multiple of
// it) -- and 32 TN output channels.  Needs the reduction channels to be a
// multiple of 16.
// ---------------------------------------------------------------------------
constexpr int conv_block_pix(int tm) { return 128 * tm; }
// largest staged region over the allowed widths: (pixels / w + 2) rows of w + 2
constexpr int conv_halo_pix(int bp) {
  int m = 0;
  for (int w = 16; w <= 256; w *= 2) {
    const int v = (bp / w + 2) * (w + 2);
    if (bp % w == 0 && v > m) m = v;
  }
  return m;
}

template <int TM, int TN>
__global__ __launch_bounds__(256) void conv3x3_lds(GemmArgs a) {
  constexpr int BP = conv_block_pix(TM), BC = 32 * TN;
  __shared__ uint4 sA[conv_halo_pix(BP) * 2];  // [region pixel][channel half of the group]
  __shared__ uint4 sB[BC * 9 * 2];             // [output channel][tap][channel half]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5;
  const int w = a.w, h = a.h, rw = w + 2;
  const int64_t p0 = (int64_t)blockIdx.x * BP;
  const int img = (int)(p0 / ((int64_t)h * w));
  const int y0 = (int)((p0 - (int64_t)img * h * w) / w);  // first image row of the block
  const int rows = BP / w + 2;                            // staged rows, halo included
  const int col0 = blockIdx.y * BC;
  const int64_t img_base = (int64_t)img * h * w;
  floatx16 acc[TM][TN];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[t][u] = floatx16{};
  // this lane's pixels within the block (row-major over the block's rows)
  int pr[TM], pc[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const int q = wave * 32 * TM + 32 * t + (lane & 31);
    pr[t] = q / w;
    pc[t] = q - pr[t] * w;
  }
  // Software pipeline over the 16-channel groups: the next group's global
  // loads go to registers before this group's taps run, and are parked in
  // LDS after the barrier that ends them.  Each thread's staged elements
  // keep their place from group to group; only the channel offset moves.
  constexpr int KA = (conv_halo_pix(BP) * 2 + 255) / 256, KB = (BC * 9 * 2 + 255) / 256;
  const int nA = rows * rw * 2;
  constexpr uint32_t kNone = 0xffffffffu;  // element outside the image or the weights
  uint32_t offA[KA], offB[KB];              // element offsets (host keeps them below 2^32 - 1)
#pragma unroll
  for (int i = 0; i < KA; ++i) {
    const int e = tid + 256 * i, q = e >> 1, hf = e & 1;
    const int ry = q / rw, rx = q - ry * rw;
    const int y = y0 - 1 + ry, x = rx - 1;
    offA[i] = (e < nA && y >= 0 && y < h && x >= 0 && x < w)
                  ? (uint32_t)((img_base + (int64_t)y * w + x) * a.x_cs + a.x_co + 8 * hf)
                  : kNone;
  }
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int e = tid + 256 * i, co = e / 18, rem = e - co * 18;
    const int tap = rem >> 1, hf = rem & 1;
    offB[i] = (e < BC * 9 * 2 && col0 + co < a.nout) ? (uint32_t)(((int64_t)(col0 + co) * 9 + tap) * a.kc + 8 * hf)
                                                     : kNone;
  }
  uint4 ra[KA], rb[KB];
  auto fetch = [&](int ch) {
#pragma unroll
    for (int i = 0; i < KA; ++i)
      ra[i] = offA[i] != kNone ? *reinterpret_cast<const uint4 *>(a.x + offA[i] + ch) : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < KB; ++i)
      rb[i] = offB[i] != kNone ? *reinterpret_cast<const uint4 *>(a.wgt + offB[i] + ch) : make_uint4(0, 0, 0, 0);
  };
  const int groups = a.kc / 16;
  fetch(0);
  for (int g = 0; g < groups; ++g) {
#pragma unroll
    for (int i = 0; i < KA; ++i)
      if (tid + 256 * i < nA) sA[tid + 256 * i] = ra[i];
#pragma unroll
    for (int i = 0; i < KB; ++i)
      if (tid + 256 * i < BC * 9 * 2) sB[tid + 256 * i] = rb[i];
    __syncthreads();
    if (g + 1 < groups) fetch((g + 1) * 16);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;
      bf16x8 A[TM], B[TN];
#pragma unroll
      for (int t = 0; t < TM; ++t)
        A[t] = __builtin_bit_cast(bf16x8, sA[((pr[t] + dy) * rw + pc[t] + dx) * 2 + half]);
#pragma unroll
      for (int u = 0; u < TN; ++u)
        B[u] = __builtin_bit_cast(bf16x8, sB[((32 * u + (lane & 31)) * 9 + tap) * 2 + half]);
#pragma unroll
      for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int u = 0; u < TN; ++u) acc[t][u] = mfma(A[t], B[u], acc[t][u]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int col = col0 + 32 * u + (lane & 31);
    if (col >= a.nout) continue;
    const float bv = a.bias ? a.bias[col] : 0.f;
#pragma unroll
    for (int t = 0; t < TM; ++t) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t p = p0 + wave * 32 * TM + 32 * t + c_row(r, lane);
        float v = acc[t][u][r] + bv;
        if (a.relu) v = v > 0.f ? v : 0.f;
        a.y[p * a.y_cs + a.y_co + col] = f2bf(v);
      }
    }
  }
}

// Can the LDS-staged kernel with block of bp pixels run this convolution?
static bool conv_lds_fits(const GemmArgs &a, int bp) {
  // element offsets of the input and the weights must fit 32 bits
  const bool small = (int64_t)a.n * a.h * a.w * a.x_cs < ((int64_t)1 << 32) - 1 &&
                     (int64_t)a.nout * 9 * a.kc < ((int64_t)1 << 32) - 1;
  return small && a.kc % 16 == 0 && a.w >= 16 && a.w <= 256 && bp % a.w == 0 &&
         ((int64_t)a.h * a.w) % bp == 0;
}

// Launch with the wave tile chosen by the output channel count.
template <int MODE>
static void launch_igemm(const GemmArgs &a, int64_t P, int taps_z, hipStream_t s) {
  if (MODE == 0 && a.nout <= 32 && conv_lds_fits(a, conv_block_pix(4))) {
    dim3 g((unsigned)(P / conv_block_pix(4)), 1);
    conv3x3_lds<4, 1><<<g, 256, 0, s>>>(a);
    return;
  }
  if (MODE == 0 && conv_lds_fits(a, conv_block_pix(2))) {
    dim3 g((unsigned)(P / conv_block_pix(2)), (unsigned)((a.nout + 63) / 64));
    conv3x3_lds<2, 2><<<g, 256, 0, s>>>(a);
    return;
  }
  if (a.nout >= 64) {
    dim3 g((unsigned)((P + 255) / 256), (unsigned)((a.nout + 63) / 64), (unsigned)taps_z);
    igemm_fwd<MODE, 2, 2><<<g, 256, 0, s>>>(a);
  } else {
    dim3 g((unsigned)((P + 511) / 512), (unsigned)((a.nout + 31) / 32), (unsigned)taps_z);
    igemm_fwd<MODE, 4, 1><<<g, 256, 0, s>>>(a);
  }
}

// ---------------------------------------------------------------------------
// Weight gradients (split over pixels): partial[kb][m][n] = sum over this
// block's pixel chunk of A(m, p) B(p, n).
//   MODE 0, 3x3: m = co, n = (tap, ci): A = dy[p][co], B = x[p + off(tap)][ci]
//   MODE 1, transposed 2x2, tap = blockIdx.z: m = co, n = ci:
//          A = dy[2p + tap][co], B = x[p][ci]  (p over the input grid)
// Per stage of 128 pixels, each thread loads an 8-pixel x 8-channel block of
// one operand (eight 16-byte vectors), transposes it in registers (byte
// permutes) and writes it channel-major to LDS as eight 16-byte vectors, so
// an MFMA operand fragment (8 consecutive pixels of one channel) is one
// 128-bit LDS read and neither side of LDS sees bank conflicts.  Channel
// counts, strides and offsets are multiples of 8.
// ---------------------------------------------------------------------------
constexpr int kWgradPix = 4096;  // pixels per block (split-K chunk)
constexpr int kStagePix = 128;   // pixels per LDS stage
constexpr int kStageLd = kStagePix + 8;

struct WgradArgs {
  const uint16_t *x;
  int n, h, w, cin, x_cs, x_co;   // x grid (input grid for MODE 1)
  const uint16_t *dy;
  int cout, dy_cs, dy_co;
  float *partial;                 // [kblocks][ntap][cout][ncol]
  int ncol;                       // MODE 0: 9 * cin; MODE 1: cin
  float *bpartial;                // [kblocks][ntap][cout] bias partial sums, or NULL
};

// 8 x 8 transpose of 16-bit values: in[p] holds channels 0..7 of pixel p,
// out[c] receives pixels 0..7 of channel c.
__device__ __forceinline__ void transpose8x8(const uint4 (&in)[8], uint4 (&out)[8]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t lo[4], hi[4];  // channel 2j and 2j + 1, pixel pairs i
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t a = (&in[2 * i].x)[j], b = (&in[2 * i + 1].x)[j];
      lo[i] = __builtin_amdgcn_perm(b, a, 0x05040100u);
      hi[i] = __builtin_amdgcn_perm(b, a, 0x07060302u);
    }
    out[2 * j] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    out[2 * j + 1] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
  }
}

// Block tile (32 MT) x (32 NT) of C with MT * NT = 4 waves, each one 32 x 32
// MFMA tile: (2, 2) in general, (1, 4) when the output channels fit 32.
template <int MODE, int MT, int NT>
__global__ __launch_bounds__(256) void igemm_wgrad(WgradArgs a) {
  static_assert(MT * NT == 4, "four waves");
  __shared__ __attribute__((aligned(16))) uint16_t sA[32 * MT][kStageLd];  // [m][pixel]
  __shared__ __attribute__((aligned(16))) uint16_t sB[32 * NT][kStageLd];  // [n][pixel]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % MT, wn = wave / MT;
  const int half = lane >> 5;
  const int64_t P = (int64_t)a.n * a.h * a.w;
  const int64_t p_begin = (int64_t)blockIdx.x * kWgradPix;
  const int m0 = blockIdx.y * 32 * MT;  // output channel block
  const int tapz = MODE == 1 ? (int)(blockIdx.z % 4) : 0;
  const int nblk = MODE == 1 ? (int)(blockIdx.z / 4) : (int)blockIdx.z;
  const int n0 = nblk * 32 * NT;        // column block
  floatx16 acc = {};
  // the blocks of the first column block also sum dy over their pixels (bias)
  const bool bias_blk = a.bpartial && nblk == 0 && tid < 32 * MT;
  float bacc = 0.f;
  const int64_t p_end = p_begin + kWgradPix < P ? p_begin + kWgradPix : P;
  // staging: 8-pixel x 8-channel blocks, 64 MT of A then 64 NT of B; a
  // thread owns entries tid and tid + 256.  The next stage's loads go to
  // registers before this stage's products run; the transpose and the LDS
  // stores follow the barrier that ends them.
  constexpr int kEntries = 64 * (MT + NT), NE = (kEntries + 255) / 256;
  uint4 v[NE][8];
  auto load_stage = [&](int64_t pcs) {
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const int e = tid + 256 * j;
      const bool stage_b = e >= 64 * MT;
      const int eo = stage_b ? e - 64 * MT : e;
      const int cg = eo >> 4, pb = eo & 15;
      // image, row and column of the first of the 8 consecutive pixels; the
      // others follow by increments (wrapping at row and image ends)
      const int64_t pfirst = pcs + pb * 8;
      int pn = (int)(pfirst / ((int64_t)a.h * a.w));
      const int rr0 = (int)(pfirst - (int64_t)pn * a.h * a.w);
      int py = rr0 / a.w, px = rr0 - py * a.w;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t p = pfirst + r;
        if (r > 0 && ++px == a.w) {
          px = 0;
          if (++py == a.h) {
            py = 0;
            ++pn;
          }
        }
        v[j][r] = make_uint4(0, 0, 0, 0);
        if (e >= kEntries || p >= p_end) continue;
        if (!stage_b) {
          const int m = m0 + cg * 8;
          if (m < a.cout) {
            int64_t q;
            if constexpr (MODE == 0) {
              q = p;
            } else {
              const int H2 = 2 * a.h, W2 = 2 * a.w;
              q = (int64_t)pn * H2 * W2 + (int64_t)(2 * py + (tapz >> 1)) * W2 + 2 * px + (tapz & 1);
            }
            v[j][r] = *reinterpret_cast<const uint4 *>(a.dy + q * a.dy_cs + a.dy_co + m);
          }
        } else {
          const int nn = n0 + cg * 8;
          if (nn < a.ncol) {
            if constexpr (MODE == 0) {
              const int tap = nn / a.cin, ci = nn - tap * a.cin;
              const int yy = py + tap / 3 - 1, xx = px + tap % 3 - 1;
              if (yy >= 0 && yy < a.h && xx >= 0 && xx < a.w)
                v[j][r] = *reinterpret_cast<const uint4 *>(
                    a.x + ((int64_t)pn * a.h * a.w + (int64_t)yy * a.w + xx) * a.x_cs + a.x_co + ci);
            } else {
              v[j][r] = *reinterpret_cast<const uint4 *>(a.x + p * a.x_cs + a.x_co + nn);
            }
          }
        }
      }
    }
  };
  if (p_begin < p_end) load_stage(p_begin);
  for (int64_t pc = p_begin; pc < p_end; pc += kStagePix) {
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const int e = tid + 256 * j;
      if (e >= kEntries) continue;
      const bool stage_b = e >= 64 * MT;
      const int eo = stage_b ? e - 64 * MT : e;
      const int cg = eo >> 4, pb = eo & 15;
      uint4 t[8];
      transpose8x8(v[j], t);
      uint16_t(*dst)[kStageLd] = stage_b ? sB : sA;
#pragma unroll
      for (int c = 0; c < 8; ++c) *reinterpret_cast<uint4 *>(&dst[cg * 8 + c][pb * 8]) = t[c];
    }
    __syncthreads();
    if (pc + kStagePix < p_end) load_stage(pc + kStagePix);
    if (bias_blk) {
#pragma unroll
      for (int q = 0; q < kStagePix; q += 8) {
        const uint4 u = *reinterpret_cast<const uint4 *>(&sA[tid][q]);
        const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) bacc += bf2f((uint16_t)(w4[k] & 0xffffu)) + bf2f((uint16_t)(w4[k] >> 16));
      }
    }
#pragma unroll
    for (int ks = 0; ks < kStagePix; ks += 16) {
      const uint4 av = *reinterpret_cast<const uint4 *>(&sA[wm * 32 + (lane & 31)][ks + 8 * half]);
      const uint4 bv = *reinterpret_cast<const uint4 *>(&sB[wn * 32 + (lane & 31)][ks + 8 * half]);
      acc = mfma(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), acc);
    }
    __syncthreads();
  }
  const int ntap = MODE == 1 ? 4 : 1;
  if (bias_blk && m0 + tid < a.cout)
    a.bpartial[((int64_t)blockIdx.x * ntap + tapz) * a.cout + m0 + tid] = bacc;
  const int nn = n0 + wn * 32 + (lane & 31);
  if (nn >= a.ncol) return;
  float *out = a.partial + ((int64_t)blockIdx.x * ntap + tapz) * (int64_t)a.cout * a.ncol;
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + wm * 32 + c_row(r, lane);
    if (m < a.cout) out[(int64_t)m * a.ncol + nn] = acc[r];
  }
}

// sum_{k < count} p[k * stride] in a fixed order: eight interleaved partial
// sums (k mod 8) combined pairwise, so the loads of a thread overlap.
__device__ __forceinline__ float strided_sum(const float *p, int64_t count, int64_t stride) {
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int64_t k = 0;
  for (; k + 8 <= count; k += 8)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] += p[(k + j) * stride];
  for (int j = 0; k + j < count; ++j) acc[j] += p[(k + j) * stride];
  return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// dw[m][tap][n] (+)= sum over kblocks of partial[kb][tap][m][n], fixed order.
// For MODE 0 ntap = 1 and n = (tap, ci) already.
__global__ void wgrad_reduce(const float *partial, int kblocks, int ntap, int cout, int ncol, float *dw,
                             int accumulate) {
  const int64_t total = (int64_t)ntap * cout * ncol;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int tap = (int)(e / ((int64_t)cout * ncol));
    const int64_t rem = e - (int64_t)tap * cout * ncol;
    const int m = (int)(rem / ncol), n = (int)(rem - (int64_t)m * ncol);
    const float s = strided_sum(partial + e, kblocks, total);
    const int64_t o = ((int64_t)m * ntap + tap) * ncol + n;  // [co][tap][ci]
    dw[o] = accumulate ? dw[o] + s : s;
  }
}

// db[c] (+)= sum over the weight-gradient blocks' bias partials, fixed order.
__global__ void bias_reduce(const float *bpartial, int64_t nparts, int c, float *db, int accumulate) {
  const int ch = blockIdx.x * blockDim.x + threadIdx.x;
  if (ch >= c) return;
  const float s = strided_sum(bpartial + ch, nparts, c);
  db[ch] = accumulate ? db[ch] + s : s;
}


// wt[ci][ky][kx][co] = w[co][2-ky][2-kx][ci]
__global__ void conv_flip(const uint16_t *w, int cout, int cin, uint16_t *wt) {
  const int64_t total = (int64_t)cout * 9 * cin;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int co = (int)(e / (9 * cin));
    const int r = (int)(e - (int64_t)co * 9 * cin);
    const int tap = r / cin, ci = r - tap * cin;
    wt[((int64_t)ci * 9 + (8 - tap)) * cout + co] = w[e];
  }
}

// wt[ci][tap][co] = w[co][tap][ci] (2x2 taps)
__global__ void up_rearrange(const uint16_t *w, int cout, int cin, uint16_t *wt) {
  const int64_t total = (int64_t)cout * 4 * cin;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int co = (int)(e / (4 * cin));
    const int r = (int)(e - (int64_t)co * 4 * cin);
    const int tap = r / cin, ci = r - tap * cin;
    wt[((int64_t)ci * 4 + tap) * cout + co] = w[e];
  }
}

__global__ void relu_bwd_kernel(const uint16_t *y, int64_t n_pix, int c, int y_cs, int y_co, uint16_t *dy,
                                int dy_cs, int dy_co) {
  const int64_t total = n_pix * c;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / c;
    const int ch = (int)(e - p * c);
    if (!(bf2f(y[p * y_cs + y_co + ch]) > 0.f)) dy[p * dy_cs + dy_co + ch] = 0;
  }
}

__global__ void maxpool_fwd_kernel(const uint16_t *x, int n, int h, int w, int c, int x_cs, int x_co, uint16_t *y,
                                   int y_cs, int y_co) {
  const int h2 = h / 2, w2 = w / 2;
  const int64_t total = (int64_t)n * h2 * w2 * c;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int ch = (int)(e % c);
    const int64_t q = e / c;
    const int qn = (int)(q / ((int64_t)h2 * w2));
    const int r = (int)(q - (int64_t)qn * h2 * w2);
    const int qy = r / w2, qx = r - qy * w2;
    float m = -INFINITY;
    uint16_t best = 0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const uint16_t v = x[((int64_t)qn * h * w + (int64_t)(2 * qy + a) * w + 2 * qx + b) * x_cs + x_co + ch];
        if (bf2f(v) > m) { m = bf2f(v); best = v; }
      }
    y[q * y_cs + y_co + ch] = best;
  }
}

// Vector form (channel counts, strides and offsets multiples of 8): one
// 16-byte vector of 8 channels per thread.
__global__ void relu_bwd_vec(const uint16_t *y, int64_t n_pix, int c8, int y_cs, int y_co, uint16_t *dy, int dy_cs,
                             int dy_co) {
  const int64_t total = n_pix * c8;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / c8;
    const int ch = (int)(e - p * c8) * 8;
    const uint4 yv = *reinterpret_cast<const uint4 *>(y + p * y_cs + y_co + ch);
    uint4 *dp = reinterpret_cast<uint4 *>(dy + p * dy_cs + dy_co + ch);
    uint4 g = *dp;
    const uint32_t yy[4] = {yv.x, yv.y, yv.z, yv.w};
    uint32_t gg[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!(bf2f((uint16_t)(yy[k] & 0xffffu)) > 0.f)) gg[k] &= 0xffff0000u;
      if (!(bf2f((uint16_t)(yy[k] >> 16)) > 0.f)) gg[k] &= 0x0000ffffu;
    }
    *dp = make_uint4(gg[0], gg[1], gg[2], gg[3]);
  }
}

__global__ void maxpool_bwd_kernel(const uint16_t *x, int n, int h, int w, int c, int x_cs, int x_co,
                                   const uint16_t *dy, int dy_cs, int dy_co, uint16_t *dx, int dx_cs, int dx_co,
                                   int accumulate) {
  const int h2 = h / 2, w2 = w / 2;
  const int64_t total = (int64_t)n * h2 * w2 * c;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int ch = (int)(e % c);
    const int64_t q = e / c;
    const int qn = (int)(q / ((int64_t)h2 * w2));
    const int r = (int)(q - (int64_t)qn * h2 * w2);
    const int qy = r / w2, qx = r - qy * w2;
    float m = -INFINITY;
    int arg = 0;
    for (int k = 0; k < 4; ++k) {
      const float v = bf2f(x[((int64_t)qn * h * w + (int64_t)(2 * qy + k / 2) * w + 2 * qx + k % 2) * x_cs + x_co + ch]);
      if (v > m) { m = v; arg = k; }
    }
    const uint16_t g = dy[q * dy_cs + dy_co + ch];
    for (int k = 0; k < 4; ++k) {
      uint16_t *d = dx + ((int64_t)qn * h * w + (int64_t)(2 * qy + k / 2) * w + 2 * qx + k % 2) * dx_cs + dx_co + ch;
      if (accumulate) {
        if (k == arg) *d = f2bf(bf2f(*d) + bf2f(g));
      } else {
        *d = k == arg ? g : 0;
      }
    }
  }
}

__device__ __forceinline__ float head_logit(const uint16_t *x, int64_t p, int c, int x_cs, const float *w, float b) {
  float z = b;
  if ((c & 7) == 0 && (x_cs & 7) == 0) {  // 16-byte vectors of 8 channels
    for (int c8 = 0; c8 < c; c8 += 8) {
      const uint4 v = *reinterpret_cast<const uint4 *>(x + p * x_cs + c8);
      const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        z += w[c8 + 2 * k] * bf2f((uint16_t)(u[k] & 0xffffu));
        z += w[c8 + 2 * k + 1] * bf2f((uint16_t)(u[k] >> 16));
      }
    }
    return z;
  }
  for (int ch = 0; ch < c; ++ch) z += w[ch] * bf2f(x[p * x_cs + ch]);
  return z;
}

__global__ void head_fwd_kernel(const uint16_t *x, int64_t n_pix, int c, int x_cs, const float *w, const float *b,
                                float *sat) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n_pix; p += (int64_t)gridDim.x * blockDim.x)
    sat[p] = 1.f / (1.f + __expf(-head_logit(x, p, c, x_cs, w, b[0])));
}

// Per pixel: logit z, loss term l = softplus(z) - t z (binary cross-entropy
// written on the logit), gradient g = (sigmoid(z) - t) * scale on masked
// pixels (0 elsewhere), and dx = g w.  g and l go to scratch for the sums.
__global__ void head_loss_pix(const uint16_t *x, int64_t n_pix, int c, int x_cs, const float *w, const float *b,
                              const float *t, const uint8_t *mask, float scale, uint16_t *dx, float *g_out,
                              float *l_out) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n_pix; p += (int64_t)gridDim.x * blockDim.x) {
    const float z = head_logit(x, p, c, x_cs, w, b[0]);
    const bool on = mask[p] != 0;
    const float sp = fmaxf(z, 0.f) + log1pf(__expf(-fabsf(z)));
    const float s = 1.f / (1.f + __expf(-z));
    const float g = on ? (s - t[p]) * scale : 0.f;
    g_out[p] = g;
    l_out[p] = on ? (sp - t[p] * z) * scale : 0.f;
    if (dx && (c & 7) == 0) {
      for (int c8 = 0; c8 < c; c8 += 8) {
        uint32_t u[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          u[k] = (uint32_t)f2bf(g * w[c8 + 2 * k]) | ((uint32_t)f2bf(g * w[c8 + 2 * k + 1]) << 16);
        *reinterpret_cast<uint4 *>(dx + p * c + c8) = make_uint4(u[0], u[1], u[2], u[3]);
      }
    } else if (dx) {
      for (int ch = 0; ch < c; ++ch) dx[p * c + ch] = f2bf(g * w[ch]);
    }
  }
}

// Block partials over a pixel chunk: threads = (256 / c) pixel lanes x c
// channels.  out[block] = {sum l, sum g, sum g x[.][0..c)}.
constexpr int kHeadPix = 4096;
__global__ void head_loss_sums(const uint16_t *x, int64_t n_pix, int c, int x_cs, const float *g, const float *l,
                               float *partial) {
  __shared__ float red[256];
  __shared__ float red_l[256], red_g[256];
  const int lanes = 256 / c;
  const int pl = threadIdx.x / c, ch = threadIdx.x - pl * c;
  const int64_t p0 = (int64_t)blockIdx.x * kHeadPix;
  float a = 0.f, sl = 0.f, sg = 0.f;
  for (int k = pl; k < kHeadPix; k += lanes) {
    const int64_t p = p0 + k;
    if (p >= n_pix) break;
    a += g[p] * bf2f(x[p * x_cs + ch]);
    if (ch == 0) { sl += l[p]; sg += g[p]; }
  }
  red[threadIdx.x] = a;
  red_l[threadIdx.x] = sl;
  red_g[threadIdx.x] = sg;
  __syncthreads();
  if (threadIdx.x < (unsigned)c) {
    float s = 0.f;
    for (int q = 0; q < lanes; ++q) s += red[q * c + threadIdx.x];
    partial[(int64_t)blockIdx.x * (2 + c) + 2 + threadIdx.x] = s;
  }
  if (threadIdx.x == 0) {
    float s1 = 0.f, s2 = 0.f;
    for (int q = 0; q < lanes; ++q) { s1 += red_l[q * c]; s2 += red_g[q * c]; }
    partial[(int64_t)blockIdx.x * (2 + c)] = s1;
    partial[(int64_t)blockIdx.x * (2 + c) + 1] = s2;
  }
}

// Vector form of head_loss_sums (c and x_cs multiples of 8): threads =
// (256 / (c / 8)) pixel lanes x (c / 8) channel groups of eight, each with
// eight accumulators fed by one 16-byte load per pixel.
__global__ void head_loss_sums_v(const uint16_t *x, int64_t n_pix, int c, int x_cs, const float *g, const float *l,
                                 float *partial) {
  __shared__ float red[256 * 8];
  __shared__ float red_l[256], red_g[256];
  const int groups = c / 8, lanes = 256 / groups;
  const int pl = threadIdx.x / groups, cg = threadIdx.x - pl * groups;
  const int64_t p0 = (int64_t)blockIdx.x * kHeadPix;
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float sl = 0.f, sg = 0.f;
  for (int k = pl; k < kHeadPix; k += lanes) {
    const int64_t p = p0 + k;
    if (p >= n_pix) break;
    const float gv = g[p];
    const uint4 v = *reinterpret_cast<const uint4 *>(x + p * x_cs + cg * 8);
    const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[2 * q] += gv * bf2f((uint16_t)(u[q] & 0xffffu));
      a[2 * q + 1] += gv * bf2f((uint16_t)(u[q] >> 16));
    }
    if (cg == 0) { sl += l[p]; sg += gv; }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) red[threadIdx.x * 8 + j] = a[j];
  red_l[threadIdx.x] = sl;
  red_g[threadIdx.x] = sg;
  __syncthreads();
  if (threadIdx.x < (unsigned)c) {
    const int ch = threadIdx.x, g8 = ch >> 3, j = ch & 7;
    float s = 0.f;
    for (int q = 0; q < lanes; ++q) s += red[(q * groups + g8) * 8 + j];
    partial[(int64_t)blockIdx.x * (2 + c) + 2 + ch] = s;
  }
  if (threadIdx.x == 0) {
    float s1 = 0.f, s2 = 0.f;
    for (int q = 0; q < lanes; ++q) { s1 += red_l[q * groups]; s2 += red_g[q * groups]; }
    partial[(int64_t)blockIdx.x * (2 + c)] = s1;
    partial[(int64_t)blockIdx.x * (2 + c) + 1] = s2;
  }
}

__global__ void head_loss_final(const float *partial, int blocks, int c, float *loss, float *dw, float *db) {
  const int k = threadIdx.x;
  if (k >= 2 + c) return;
  const float s = strided_sum(partial + k, blocks, 2 + c);
  if (k == 0) loss[0] = s;
  else if (k == 1) { if (db) db[0] = s; }
  else if (dw) dw[k - 2] = s;
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = f2bf(pi);
  }
}

__global__ void to_bf16_kernel(const float *x, uint16_t *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = f2bf(x[i]);
}
__global__ void to_f32_kernel(const uint16_t *x, float *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = bf2f(x[i]);
}

static int grid1d(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}
static int launched() { return hipGetLastError() == hipSuccess ? 0 : -100; }
static bool ok8(int v) { return v > 0 && v % 8 == 0; }

}  // namespace unet

using namespace unet;

// Split-K partial sums of the allocation-free weight gradient: a file-scope
// device array, one copy per GPU, held until the process ends.  Host code
// never uses its name as an address: the address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr int64_t kStaticScratchFloats = (int64_t)4 << 20;  // 16 MiB
static __device__ __align__(256) float scratch[kStaticScratchFloats];

static float *scratch_ptr_current_device() {
  static std::mutex mu;
  static float *ptrs[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    ptrs[dev] = static_cast<float *>(p);
  }
  return ptrs[dev];
}

// A channel slice [co, co + c) of a tensor with cs channels per pixel lies
// inside the tensor.
static bool slice_ok(int co, int c, int cs) { return co >= 0 && c >= 1 && (int64_t)co + c <= cs; }

extern "C" {

int unet_mfma_probe(const uint16_t *A, const uint16_t *B, float *C, void *s) {
  mfma_probe_kernel<<<1, 64, 0, (hipStream_t)s>>>(A, B, C);
  return launched();
}

int unet_conv3x3_fwd(const uint16_t *x, int n, int h, int w, int cin, int x_cs, int x_co, const uint16_t *wgt,
                     const float *bias, int cout, uint16_t *y, int y_cs, int y_co, int relu, void *s) {
  if (!x || !wgt || !y || n < 1 || h < 1 || w < 1 || !ok8(cin) || x_cs % 8 || x_co % 8 ||
      !slice_ok(x_co, cin, x_cs) || !slice_ok(y_co, cout, y_cs))
    return -1;
  GemmArgs a{x, n, h, w, cin, x_cs, x_co, wgt, bias, cout, y, y_cs, y_co, relu};
  launch_igemm<0>(a, (int64_t)n * h * w, 1, (hipStream_t)s);
  return launched();
}

int unet_conv3x3_flip(const uint16_t *wgt, int cout, int cin, uint16_t *wt, void *s) {
  if (!wgt || !wt || cout < 1 || cin < 1) return -1;
  conv_flip<<<grid1d((int64_t)cout * 9 * cin), 256, 0, (hipStream_t)s>>>(wgt, cout, cin, wt);
  return launched();
}

int64_t unet_wgrad_scratch_floats(int n, int h, int w, int cin, int cout, int taps) {
  const int64_t P = (int64_t)n * h * w;
  const int64_t kb = (P + kWgradPix - 1) / kWgradPix;
  const int64_t wpart = kb * (int64_t)cout * cin * taps;
  const int64_t bpart = kb * (taps == 4 ? 4 : 1) * (int64_t)cout;  // bias partials follow
  return wpart + bpart;
}

int unet_conv3x3_wgrad(const uint16_t *x, int n, int h, int w, int cin, int x_cs, int x_co, const uint16_t *dy,
                       int cout, int dy_cs, int dy_co, float *dw, float *db, float *partial, int accumulate,
                       void *s) {
  if (!x || !dy || !dw || !partial || n < 1 || h < 1 || w < 1 || !ok8(cin) || !ok8(cout) || x_cs % 8 ||
      x_co % 8 || dy_cs % 8 || dy_co % 8 || x_co + cin > x_cs || dy_co + cout > dy_cs)
    return -1;
  const int64_t P = (int64_t)n * h * w;
  const int kb = (int)((P + kWgradPix - 1) / kWgradPix);
  const int64_t wpart = (int64_t)kb * cout * 9 * cin;
  WgradArgs a{x, n, h, w, cin, x_cs, x_co, dy, cout, dy_cs, dy_co, partial, 9 * cin, db ? partial + wpart : nullptr};
  if (cout <= 32) {
    dim3 g((unsigned)kb, 1, (unsigned)((9 * cin + 127) / 128));
    igemm_wgrad<0, 1, 4><<<g, 256, 0, (hipStream_t)s>>>(a);
  } else {
    dim3 g((unsigned)kb, (unsigned)((cout + 63) / 64), (unsigned)((9 * cin + 63) / 64));
    igemm_wgrad<0, 2, 2><<<g, 256, 0, (hipStream_t)s>>>(a);
  }
  wgrad_reduce<<<grid1d((int64_t)cout * 9 * cin), 256, 0, (hipStream_t)s>>>(partial, kb, 1, cout, 9 * cin, dw,
                                                                             accumulate);
  if (db) bias_reduce<<<(cout + 63) / 64, 64, 0, (hipStream_t)s>>>(partial + wpart, kb, cout, db, accumulate);
  return launched();
}

int unet_conv3x3_wgrad_noalloc(const uint16_t *x, int n, int h, int w, int cin, int x_cs, int x_co,
                               const uint16_t *dy, int cout, int dy_cs, int dy_co, float *dw, float *db,
                               int accumulate, void *s) {
  if (!x || !dy || !dw || n < 1 || h < 1 || w < 1 || !ok8(cin) || !ok8(cout) || x_cs % 8 || x_co % 8 ||
      dy_cs % 8 || dy_co % 8 || !slice_ok(x_co, cin, x_cs) || !slice_ok(dy_co, cout, dy_cs))
    return -1;
  if (unet_wgrad_scratch_floats(n, h, w, cin, cout, 9) > kStaticScratchFloats) return -2;
  float *part = scratch_ptr_current_device();
  if (!part) return -100;
  return unet_conv3x3_wgrad(x, n, h, w, cin, x_cs, x_co, dy, cout, dy_cs, dy_co, dw, db, part, accumulate, s);
}

int unet_relu_bwd(const uint16_t *y, int n_pix, int c, int y_cs, int y_co, uint16_t *dy, int dy_cs, int dy_co,
                  void *s) {
  if (!y || !dy || n_pix < 1 || !slice_ok(y_co, c, y_cs) || !slice_ok(dy_co, c, dy_cs)) return -1;
  if (c % 8 == 0 && y_cs % 8 == 0 && y_co % 8 == 0 && dy_cs % 8 == 0 && dy_co % 8 == 0)
    relu_bwd_vec<<<grid1d((int64_t)n_pix * (c / 8)), 256, 0, (hipStream_t)s>>>(y, n_pix, c / 8, y_cs, y_co, dy,
                                                                                dy_cs, dy_co);
  else
    relu_bwd_kernel<<<grid1d((int64_t)n_pix * c), 256, 0, (hipStream_t)s>>>(y, n_pix, c, y_cs, y_co, dy, dy_cs,
                                                                            dy_co);
  return launched();
}

int unet_maxpool_fwd(const uint16_t *x, int n, int h, int w, int c, int x_cs, int x_co, uint16_t *y, int y_cs,
                     int y_co, void *s) {
  if (!x || !y || n < 1 || h < 2 || w < 2 || (h & 1) || (w & 1) || !slice_ok(x_co, c, x_cs) ||
      !slice_ok(y_co, c, y_cs))
    return -1;
  maxpool_fwd_kernel<<<grid1d((int64_t)n * h * w * c / 4), 256, 0, (hipStream_t)s>>>(x, n, h, w, c, x_cs, x_co, y,
                                                                                       y_cs, y_co);
  return launched();
}

int unet_maxpool_bwd(const uint16_t *x, int n, int h, int w, int c, int x_cs, int x_co, const uint16_t *dy,
                     int dy_cs, int dy_co, uint16_t *dx, int dx_cs, int dx_co, int accumulate, void *s) {
  if (!x || !dy || !dx || n < 1 || h < 2 || w < 2 || (h & 1) || (w & 1) || !slice_ok(x_co, c, x_cs) ||
      !slice_ok(dy_co, c, dy_cs) || !slice_ok(dx_co, c, dx_cs))
    return -1;
  maxpool_bwd_kernel<<<grid1d((int64_t)n * h * w * c / 4), 256, 0, (hipStream_t)s>>>(
      x, n, h, w, c, x_cs, x_co, dy, dy_cs, dy_co, dx, dx_cs, dx_co, accumulate);
  return launched();
}

int unet_upconv_fwd(const uint16_t *x, int n, int h, int w, int cin, int x_cs, int x_co, const uint16_t *wgt,
                    const float *bias, int cout, uint16_t *y, int y_cs, int y_co, void *s) {
  if (!x || !wgt || !y || n < 1 || h < 1 || w < 1 || !ok8(cin) || x_cs % 8 || x_co % 8 ||
      !slice_ok(x_co, cin, x_cs) || !slice_ok(y_co, cout, y_cs))
    return -1;
  GemmArgs a{x, n, h, w, cin, x_cs, x_co, wgt, bias, cout, y, y_cs, y_co, 0};
  launch_igemm<1>(a, (int64_t)n * h * w, 4, (hipStream_t)s);
  return launched();
}

int unet_upconv_bwd_data(const uint16_t *dy, int n, int h, int w, int cout, int dy_cs, int dy_co,
                         const uint16_t *wgt, int cin, uint16_t *wt, uint16_t *dx, int dx_cs, int dx_co, void *s) {
  if (!dy || !wgt || !wt || !dx || n < 1 || h < 1 || w < 1 || !ok8(cout) || dy_cs % 8 || dy_co % 8 ||
      !slice_ok(dy_co, cout, dy_cs) || !slice_ok(dx_co, cin, dx_cs))
    return -1;
  up_rearrange<<<grid1d((int64_t)cout * 4 * cin), 256, 0, (hipStream_t)s>>>(wgt, cout, cin, wt);
  // A = dy over the 2h x 2w grid gathered at 2p + tap, output grid h x w
  GemmArgs a{dy, n, h, w, cout, dy_cs, dy_co, wt, nullptr, cin, dx, dx_cs, dx_co, 0};
  launch_igemm<2>(a, (int64_t)n * h * w, 1, (hipStream_t)s);
  return launched();
}

int unet_upconv_wgrad(const uint16_t *x, int n, int h, int w, int cin, int x_cs, int x_co, const uint16_t *dy,
                      int cout, int dy_cs, int dy_co, float *dw, float *db, float *partial, void *s) {
  if (!x || !dy || !dw || !partial || n < 1 || h < 1 || w < 1 || !ok8(cin) || !ok8(cout) || x_cs % 8 ||
      x_co % 8 || dy_cs % 8 || dy_co % 8 || x_co + cin > x_cs || dy_co + cout > dy_cs)
    return -1;
  const int64_t P = (int64_t)n * h * w;
  const int kb = (int)((P + kWgradPix - 1) / kWgradPix);
  const int64_t wpart = (int64_t)kb * 4 * cout * cin;
  WgradArgs a{x, n, h, w, cin, x_cs, x_co, dy, cout, dy_cs, dy_co, partial, cin, db ? partial + wpart : nullptr};
  if (cout <= 32) {
    dim3 g((unsigned)kb, 1, (unsigned)(4 * ((cin + 127) / 128)));
    igemm_wgrad<1, 1, 4><<<g, 256, 0, (hipStream_t)s>>>(a);
  } else {
    dim3 g((unsigned)kb, (unsigned)((cout + 63) / 64), (unsigned)(4 * ((cin + 63) / 64)));
    igemm_wgrad<1, 2, 2><<<g, 256, 0, (hipStream_t)s>>>(a);
  }
  wgrad_reduce<<<grid1d((int64_t)4 * cout * cin), 256, 0, (hipStream_t)s>>>(partial, kb, 4, cout, cin, dw, 0);
  if (db) bias_reduce<<<(cout + 63) / 64, 64, 0, (hipStream_t)s>>>(partial + wpart, (int64_t)kb * 4, cout, db, 0);
  return launched();
}

int unet_head_fwd(const uint16_t *x, int n_pix, int c, int x_cs, const float *w, const float *b, float *sat,
                  void *s) {
  if (!x || !w || !b || !sat || n_pix < 1 || c < 1 || c > 256 || 256 % c || c > x_cs) return -1;
  head_fwd_kernel<<<grid1d(n_pix), 256, 0, (hipStream_t)s>>>(x, n_pix, c, x_cs, w, b, sat);
  return launched();
}

int64_t unet_head_scratch_floats(int n_pix, int c) {
  const int64_t blocks = ((int64_t)n_pix + kHeadPix - 1) / kHeadPix;
  return 2 * (int64_t)n_pix + blocks * (2 + c);
}

int unet_head_loss_bwd(const uint16_t *x, int n_pix, int c, int x_cs, const float *w, const float *b,
                       const float *target, const uint8_t *mask, float scale, float *loss, uint16_t *dx,
                       float *dw, float *db, float *partial, void *s) {
  if (!x || !w || !b || !target || !mask || !loss || !partial || n_pix < 1 || c < 1 || c > 256 || 256 % c ||
      c > x_cs)
    return -1;
  float *g = partial, *l = partial + n_pix, *sums = partial + 2 * (int64_t)n_pix;
  const int blocks = (int)(((int64_t)n_pix + kHeadPix - 1) / kHeadPix);
  head_loss_pix<<<grid1d(n_pix), 256, 0, (hipStream_t)s>>>(x, n_pix, c, x_cs, w, b, target, mask, scale, dx, g, l);
  if ((c & 7) == 0 && (x_cs & 7) == 0)
    head_loss_sums_v<<<blocks, 256, 0, (hipStream_t)s>>>(x, n_pix, c, x_cs, g, l, sums);
  else
    head_loss_sums<<<blocks, 256, 0, (hipStream_t)s>>>(x, n_pix, c, x_cs, g, l, sums);
  head_loss_final<<<1, 512, 0, (hipStream_t)s>>>(sums, blocks, c, loss, dw, db);
  return launched();
}

int unet_adam(float *p, const float *g, float *m, float *v, uint16_t *p_bf16, int64_t count, float lr, float beta1,
              float beta2, float eps, int step, void *s) {
  if (!p || !g || !m || !v || count < 1 || step < 1) return -1;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  adam_kernel<<<grid1d(count), 256, 0, (hipStream_t)s>>>(p, g, m, v, p_bf16, count, lr, beta1, beta2, eps, c1, c2);
  return launched();
}

int unet_to_bf16(const float *x, uint16_t *y, int64_t count, void *s) {
  if (!x || !y || count < 1) return -1;
  to_bf16_kernel<<<grid1d(count), 256, 0, (hipStream_t)s>>>(x, y, count);
  return launched();
}

int unet_to_f32(const uint16_t *x, float *y, int64_t count, void *s) {
  if (!x || !y || count < 1) return -1;
  to_f32_kernel<<<grid1d(count), 256, 0, (hipStream_t)s>>>(x, y, count);
  return launched();
}

}  // extern "C"
