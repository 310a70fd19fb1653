// Internal definitions shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm.h"

namespace lbm {

// Per-node info word.  For a fluid node, bit i (i < Q) says that the pull
// source x - e_i is solid (half-way bounce-back on link i).  For a solid node,
// bit i says that x + e_i is an in-domain fluid node (enters Eq. 17).
constexpr uint32_t kSolid = 1u << 24;
constexpr uint32_t kInlet = 1u << 25;   // fluid node at x = 0 of an open x axis
constexpr uint32_t kOutlet = 1u << 26;  // fluid node at x = nx-1 of an open x axis
constexpr uint32_t kPFace = 1u << 27;   // face node used in the boundary pressure
constexpr uint32_t kWindow = 1u << 28;  // inside the saturation window
constexpr uint32_t kLinkMask = (1u << 19) - 1u;

// 2D step tile: 64 lanes cover 60 interior columns plus 2 halo columns on
// each side; TY interior rows (8, 12 or 16) plus 2 halo rows above and below.
constexpr int kTileX = 60;
// 3D step tile: the same 64-lane rows, TY3 interior rows in y, marching in z.
constexpr int kTileY3 = 8;
// Compacted 3D fused step: a tile is one row word (64 columns) by kFwdRows
// rows, marching a chunk of z.
constexpr int kFwdRows = 8;
// Threads per block of the compacted split step's density and collision
// kernels (thread per fluid node): 128 measured 2 % faster than 256 at 384^3.
constexpr int kCompactThreads = 128;

// Compacted layout: the fluid nodes of each (y, z) row, in x order, get
// consecutive compact indices c.  A 64-node word of a row is described by its
// fluid bit mask and the compact index of its first fluid node, so the index
// of fluid node (x, row) is pre + popcount(bits below x).
struct RowWord {
  unsigned long long bits;
  long long pre;
};

// Device-side description of one instance (array in device memory).
struct InstDev {
  float *f[2];            // ping-pong post-collision state (layout by storage)
  const uint32_t *info;   // node info words, index x + pitch * (y + ny * z)
  const float *frozen;    // [2][Q][ny*nz]: component-1 outlet / component-2 inlet links
  float *psi;             // two arrays of [nz][ny][pitch] (psi1, psi2) float pairs
  const float *ivsd0;     // null, or [nz][ny][pitch] (psi1, psi2) pairs: Eq. 17 held from
                          // the initial densities (frozen reading, ivsd_frozen)
  int64_t ystride, zstride;  // f buffers: row blocks of (y, z) at y * ystride + z * zstride
  int32_t nx, ny, nz, pitch;  // pitch = padded row length (a multiple of 64)
  int32_t periodic, open_x, bc_set, collision;
  int32_t half_shift, sj_mode, storage, q;
  int32_t eq26_mode, pad_;
  int32_t tiles_x, tiles_y, tiles_z, block_base;
  double tau1, tau2, G, chi1, chi2, gx, gy, gz;
  double rho_in1, rho_out2, rho_in2, rho_out1;
  double lambda, s_e, s_eps;
  // compacted layout (compact != 0), over the compact index c (cpitch
  // entries per link): FP32 f[s][c / 64][i][c % 64]; BF16 the dense row
  // block's planes, (rho1, rho2) pairs, then deviation words
  const RowWord *cword;   // [ny * nz][pitch / 64]
  const uint32_t *ckey;   // [nf]: dense node index x + pitch * (y + ny * z) of compact node c
  const uint32_t *cinfo;  // [nf]: node info word of compact node c
  const uint32_t *cbnd;   // [nbnd]: dense index of each solid node with a fluid neighbour
  const uint32_t *cedge;  // [nedge]: compact indices of the fluid nodes whose next-step
                          // densities the compacted 3D fused step leaves to a pull
  int64_t nf, nbnd, nedge;
  int32_t cpitch, compact;
};

// Reduction record written per block by the observables kernel.
constexpr int kObsFields = 15;  // mass0 mass1 nfluid nwin swcount sumrw sumr pin nin pout nout
                                // stag_x stag_y stag_z flags

// Launchers (defined in the .hip sources).
hipError_t launch_init(const InstDev *d_inst, const InstDev &h_inst, const float *rho0_dev,
                       int parity, hipStream_t s);
hipError_t launch_ivsd_freeze(const InstDev *d_inst, const InstDev &h, int parity, hipStream_t s);
hipError_t launch_poke(const InstDev *d_inst, const InstDev &h, int parity, int x, int y, int z, int s, int i,
                       float v, int32_t *status, hipStream_t st);
// Rest equilibria of densities set from a saturation field (device, one
// float per node): (major, minor) where sat > thr, (minor, major) elsewhere.
hipError_t launch_init_sat(const InstDev *d_inst, const InstDev &h_inst, const float *sat_dev, float thr,
                           float major, float minor, int parity, hipStream_t s);
// One step of every instance of a batch.  strategy 1: fused kernel (one
// launch over a flat block table); 2: split step (three launches per instance);
// 3: compacted fluid-node step (three launches per instance, compact layout).
struct StepLaunch {
  const InstDev *d_insts;
  const InstDev *h;            // host copies (grid sizes of the split kernels)
  const int32_t *block_inst;   // fused: block -> instance table (NULL for one instance)
  const uint8_t *active;       // host flags per instance: 0 = retired, not advanced (NULL: all)
  int64_t n_blocks;            // fused: blocks of the advancing instances (may be 0)
  int k, q, collision, storage, math, strategy, ty, parity;
  bool live(int i) const { return !active || active[i]; }
};
hipError_t launch_step(const StepLaunch &L, hipStream_t s);
hipError_t launch_observables(const InstDev *d_inst, const InstDev &h_inst, int parity,
                              double *partials, int n_blocks, double *result, hipStream_t s);
hipError_t launch_density(const InstDev *d_inst, const InstDev &h_inst, int parity,
                          float *dst, hipStream_t s);
// The compacted 3D fused step carries the next step's psi between steps;
// this recomputes it from buffer `parity` (after set-up, a checkpoint load,
// a change of boundary densities or of step variant).
hipError_t launch_fwd_rebuild(const InstDev *d_inst, const InstDev &h_inst, int parity, hipStream_t s);
const char *step_kernel_name(int q, int collision, int storage, int math, int strategy, int ty);
int obs_blocks(const InstDev &h_inst);

}  // namespace lbm
