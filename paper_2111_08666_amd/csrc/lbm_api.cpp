// Host runtime behind the C ABI of include/lbm.h: argument validation, node
// tables, workspace carving, kernel launches, HIP graphs and checkpoints.
// A single-instance context is a batch of one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.h"

using namespace lbm;

namespace {

thread_local std::string g_err = "";

// host copies of the lattice tables (velocity sets of the kernels)
const int E9[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                      {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
const int E19[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                        {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                        {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                        {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
double weight(int q, int i) {
  if (q == 9) return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
const int *evec(int q, int i) { return q == 9 ? E9[i] : E19[i]; }

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }
int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct Layout {
  int32_t pitch;
  int64_t ystride, zstride, n_nodes;
  size_t buf_bytes, info_bytes, frozen_bytes, psi_bytes;
  size_t ivsd0_off;  // within the frozen block: the held Eq. 17 values (ivsd_frozen), else 0
  // compacted layout
  bool compact;
  int64_t nf, nsolid;
  int32_t cpitch;
  size_t cword_bytes, ckey_bytes, cbnd_bytes, cedge_bytes;  // cinfo: ckey_bytes
};

// Fused-kernel tiling of one instance for a tile height (D2Q9) / fixed 3D tile.
struct Tiling {
  int32_t tiles_x, tiles_y, tiles_z;
  int64_t blocks;
};

// Compute units of the device (for the z-chunking of the compacted 3D fused step).
int device_cus() {
  static int n = 0;
  if (!n) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      n = v;
    else
      n = 256;
  }
  return n;
}

Tiling make_tiling(int q, int nx, int ny, int nz, int ty, int strategy = LBM_FUSED) {
  Tiling t{};
  t.tiles_x = (nx + kTileX - 1) / kTileX;
  if (q == 19 && strategy == LBM_COMPACT_FUSED) {
    // compacted 3D fused step: tiles of one row word by kFwdRows rows, three
    // blocks resident per CU (LDS).  Choose the number of z chunks that
    // minimises (rounds of blocks) x (planes per chunk + 2): a chunk's two
    // end planes leave their densities to the edge pull.
    t.tiles_x = (nx + 63) / 64;
    t.tiles_y = (ny + kFwdRows - 1) / kFwdRows;
    const int64_t xy = (int64_t)t.tiles_x * t.tiles_y, slots = 3 * (int64_t)device_cus();
    int64_t best = -1;
    for (int tz = 1; tz <= std::max(1, nz / 8); ++tz) {
      const int64_t zlen = (nz + tz - 1) / tz;
      const int64_t cost = ((xy * tz + slots - 1) / slots) * (zlen + 2);
      if (best < 0 || cost < best) { best = cost; t.tiles_z = tz; }
    }
  } else if (q == 9) {
    t.tiles_y = (ny + ty - 1) / ty;
    t.tiles_z = 1;
  } else {
    t.tiles_y = (ny + kTileY3 - 1) / kTileY3;
    const int64_t xy = (int64_t)t.tiles_x * t.tiles_y;
    int64_t tz = (4096 + xy - 1) / xy;                  // aim at >= 4096 blocks
    tz = std::min<int64_t>(tz, std::max(1, nz / 24));  // keep z chunks >= ~24 planes
    t.tiles_z = (int32_t)std::max<int64_t>(1, tz);
  }
  t.blocks = (int64_t)t.tiles_x * t.tiles_y * t.tiles_z;
  return t;
}

// The compacted layout addresses one component's populations with 32-bit
// byte offsets (q * cpitch * 4 below 2^32), and keys each fluid node by its
// 32-bit dense index x + pitch * (y + ny * z) (pitch * ny * nz below 2^32).
bool compact_fits(const lbm_geometry &g) {
  int64_t nf = 0;
  for (int64_t n = 0; n < (int64_t)g.nx * g.ny * g.nz; ++n) nf += g.solid[n] == 0;
  const int64_t dense = round_up(g.nx, 64) * (int64_t)g.ny * g.nz;
  return (int64_t)g.q * (nf + 64) * 4 < ((int64_t)1 << 32) && dense < ((int64_t)1 << 32);
}

// The listed D2Q9 step addresses its stores as a 32-bit byte offset from the
// tile's first row: 16 row blocks of 18 pitched rows must span < 2^31 bytes.
bool list_fits(int32_t nx) { return (int64_t)16 * 18 * round_up(nx, 64) * 4 < ((int64_t)1 << 31); }

// Strategies that run on the compacted layout.
bool compact_strategy(int s) { return s == LBM_COMPACT || s == LBM_COMPACT_FUSED; }

// The step a context starts with.  Measured on MI355X: in 2D the dense fused
// kernel is fastest on the dense layout (the autotuner may still pick the
// listed variant; auto_layout below moves large batches to the compacted
// layout); in 3D the compacted layout beats the dense split step (3.7 against
// 7.7 ms per step at 384^3, porosity 0.42), since it spends nothing on solid
// nodes.
int resolve_strategy(const lbm_geometry &g, const lbm_params &p) {
  if (p.strategy != LBM_AUTO) return p.strategy;
  if (g.q == 19) return compact_fits(g) ? LBM_COMPACT : LBM_SPLIT;
  return LBM_FUSED;
}

Layout make_layout(const lbm_geometry &g, const lbm_params &p) {
  Layout L{};
  L.pitch = (int32_t)round_up(g.nx, 64);
  L.n_nodes = (int64_t)g.nx * g.ny * g.nz;
  // row block per (y, z): FP32 2Q populations; BF16 a (rho1, rho2) pair per node + Q-1 words
  // of both components' bf16 deviations (Q + 1 floats per node either way for BF16)
  L.ystride = (int64_t)(p.storage == LBM_STORE_F32 ? 2 * g.q : g.q + 1) * L.pitch;
  L.zstride = L.ystride * g.ny;
  L.buf_bytes = align_up((size_t)L.zstride * g.nz * sizeof(float));
  L.info_bytes = align_up((size_t)L.pitch * g.ny * g.nz * sizeof(uint32_t));
  // held values: Eqs. 26-27 links, then (ivsd_frozen) Eq. 17 pairs per node
  L.frozen_bytes = align_up((size_t)2 * g.q * g.ny * g.nz * sizeof(float));
  L.ivsd0_off = 0;
  if (p.ivsd_frozen) {
    L.ivsd0_off = L.frozen_bytes;
    L.frozen_bytes += align_up((size_t)L.pitch * g.ny * g.nz * 2 * sizeof(float));
  }
  L.psi_bytes = align_up((size_t)L.pitch * g.ny * g.nz * 2 * 2 * sizeof(float));  // two pair arrays
  L.compact = compact_strategy(resolve_strategy(g, p));
  if (L.compact) {  // validate() keeps q * cpitch * 4 bytes below 2^32
    int64_t nf = 0;
    for (int64_t n = 0; n < L.n_nodes; ++n) nf += g.solid[n] == 0;
    L.nf = nf;
    L.nsolid = L.n_nodes - nf;
    L.cpitch = (int32_t)round_up(std::max<int64_t>(nf, 1), 64);
    // FP32: 2Q planes; BF16: a plane of (rho1, rho2) pairs + Q-1 planes of deviation words
    L.buf_bytes = align_up((size_t)(p.storage == LBM_STORE_F32 ? 2 * g.q : g.q + 1) * L.cpitch * sizeof(float));
    L.cword_bytes = align_up((size_t)g.ny * g.nz * (L.pitch / 64) * sizeof(RowWord));
    L.ckey_bytes = align_up((size_t)std::max<int64_t>(nf, 1) * sizeof(uint32_t));
    L.cbnd_bytes = align_up((size_t)std::max<int64_t>(L.nsolid, 1) * sizeof(uint32_t));
    L.cedge_bytes = g.q == 19 ? L.ckey_bytes : 0;
  }
  return L;
}

// Rows per band of the compact numbering: `rows` if given, else chosen so
// that a 3D band's z-slice carries about 1.5 MB of population traffic (both
// components read and written), and the populations a slice leaves for its z
// neighbour slice (bounce-back reads of its own slots, pulls of the next
// slice) are still in the L2 of the XCD that walks the band.
int compact_band_rows(const lbm_geometry &g, int64_t nf, int rows) {
  if (g.nz == 1) return g.ny;
  if (rows > 0) return std::min(rows, g.ny);
  const double row_bytes = (double)nf / ((double)g.ny * g.nz) * 2.0 * 2 * g.q * sizeof(float);
  const double b = row_bytes > 0 ? 1.5e6 / row_bytes : (double)g.ny;
  return (int)std::max(1.0, std::min((double)g.ny, std::floor(b)));
}

// Compact index tables of one instance (see RowWord): row words, compact ->
// dense node index, and the solid nodes with a fluid neighbour.  Fluid nodes
// are numbered by bands of compact_band_rows() rows: band by band, in a band
// z-slice by z-slice, in a slice row by row and in a row in x order.  The
// fluid nodes of a row are therefore consecutive (what the rank arithmetic
// of the kernels needs), and a step kernel, whose threads follow the
// numbering, revisits a z-slice's populations within one slice of work
// instead of one whole plane (measured for D3Q19 at 384^3 with TRT: 30-row
// bands cut the compacted split step's L2 fetches by 20 % and its time from
// 3.38 to 3.27 ms per step; 8 to 64 rows all do about as well).  (A tile-ordered
// numbering, each kFwdRows x 64 tile plane one contiguous run, was also
// measured there: the fused 3D step gained 22 %, the compacted split step
// lost 4 %.)
void build_compact(const lbm_geometry &g, const Layout &L, const std::vector<uint32_t> &info,
                   std::vector<RowWord> &words, std::vector<uint32_t> &key, std::vector<uint32_t> &bnd,
                   int band_rows) {
  const int W = L.pitch / 64;
  const int B = compact_band_rows(g, L.nf, band_rows);
  words.assign((size_t)g.ny * g.nz * W, RowWord{0, 0});
  key.clear();
  bnd.clear();
  long long c = 0;
  for (int y0 = 0; y0 < g.ny; y0 += B)
    for (int z = 0; z < g.nz; ++z)
      for (int y = y0; y < std::min(y0 + B, g.ny); ++y) {
        const int64_t r = y + (int64_t)g.ny * z;
        for (int w = 0; w < W; ++w) {
          RowWord &rw = words[(size_t)(r * W + w)];
          rw.pre = c;
          for (int b = 0; b < 64; ++b) {
            const int x = 64 * w + b;
            if (x >= g.nx) break;
            const uint32_t dense = (uint32_t)(x + (int64_t)L.pitch * r);
            if (!g.solid[x + (int64_t)g.nx * r]) {
              rw.bits |= 1ull << b;
              key.push_back(dense);
              ++c;
            } else if (info[dense] & kLinkMask) {
              bnd.push_back(dense);
            }
          }
        }
      }
}

// FNV-1a hash of what fixes an instance's node tables (solid map, axes),
// stored in checkpoints so that a state is only restored onto its geometry.
uint64_t geometry_hash(const lbm_geometry &g) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  };
  const int32_t hd[6] = {g.q, g.nx, g.ny, g.nz, (int32_t)g.periodic, g.open_x};
  mix(hd, sizeof hd);
  mix(g.solid, (size_t)g.nx * g.ny * g.nz);
  return h;
}

bool bad(std::string &err, const std::string &msg) {
  err = msg;
  return false;
}

// Validation of one instance; no device work.
bool validate(const lbm_geometry *g, const lbm_params *p, const double *rho0, std::string &err) {
  if (!g || !p) return bad(err, "null geometry or params");
  if (g->q != 9 && g->q != 19) return bad(err, "q must be 9 or 19");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return bad(err, "grid sizes must be >= 1");
  if (g->q == 9 && g->nz != 1) return bad(err, "D2Q9 needs nz = 1");
  if ((int64_t)g->nx * g->ny * g->nz > (int64_t)1 << 31) return bad(err, "grid too large");
  if (!g->solid) return bad(err, "solid map is NULL");
  if (g->open_x && ((g->periodic & 1) || g->nx < 3)) return bad(err, "open x needs nx >= 3 and x not periodic");
  for (int c = 0; c < 2; ++c)
    if (!(p->tau[c] > 0.5) || !std::isfinite(p->tau[c])) return bad(err, "tau must exceed 1/2");
  if (!(std::fabs(p->xi) < 1.0)) return bad(err, "|xi| must be < 1");
  if (!std::isfinite(p->G)) return bad(err, "G must be finite");
  if (p->collision < 0 || p->collision > 2) return bad(err, "collision must be SRT, MRT or TRT");
  if (p->bc_set < 1 || p->bc_set > 3) return bad(err, "bc_set must be 1, 2 or 3");
  if (p->eq26_mode != 0 && p->eq26_mode != 1) return bad(err, "eq26_mode must be 0 or 1");
  if (p->ivsd_frozen != 0 && p->ivsd_frozen != 1) return bad(err, "ivsd_frozen must be 0 or 1");
  if (p->ivsd_frozen && round_up(g->nx, 64) * (int64_t)g->ny * g->nz >= ((int64_t)1 << 32))
    return bad(err, "grid too large for the held values of Eq. 17 (32-bit dense index)");
  if (p->storage != LBM_STORE_F32 && p->storage != LBM_STORE_BF16DEV) return bad(err, "unknown storage");
  if (p->math != LBM_MATH_F64 && p->math != LBM_MATH_F32) return bad(err, "unknown math precision");
  if (p->strategy < LBM_AUTO || p->strategy > LBM_COMPACT_FUSED) return bad(err, "unknown strategy");
  if (p->strategy == LBM_COMPACT_FUSED && g->q == 19 && p->storage != LBM_STORE_F32)
    return bad(err, "the compacted fused D3Q19 step needs FP32 storage");
  if (p->strategy == LBM_FUSED_LIST && g->q != 9) return bad(err, "the listed fused step is D2Q9 only");
  if (p->strategy == LBM_FUSED_LIST && !list_fits(g->nx)) return bad(err, "nx too large for the listed fused step");
  if (compact_strategy(p->strategy) && !compact_fits(*g))
    return bad(err, "too many fluid nodes for the compacted layout (use LBM_SPLIT)");
  if (p->tile_rows != 0 && p->tile_rows != 8 && p->tile_rows != 12 && p->tile_rows != 16)
    return bad(err, "tile_rows must be 0, 8, 12 or 16");
  const double vals[] = {p->rho_in1, p->rho_out2, p->rho_in2, p->rho_out1, p->g[0], p->g[1], p->g[2]};
  for (double v : vals)
    if (!std::isfinite(v)) return bad(err, "boundary densities and g must be finite");
  const int64_t N = (int64_t)g->nx * g->ny * g->nz;
  const bool perx = g->periodic & 1, pery = g->periodic & 2, perz = g->periodic & 4;
  for (int64_t n = 0; n < N; ++n) {
    if (g->solid[n]) continue;
    const int x = (int)(n % g->nx), y = (int)((n / g->nx) % g->ny), z = (int)(n / ((int64_t)g->nx * g->ny));
    int nfluid = 0;
    for (int i = 1; i < g->q; ++i) {
      const int *e = evec(g->q, i);
      int a = x + e[0], b = y + e[1], c = z + e[2];
      const bool ox = a < 0 || a >= g->nx, oy = b < 0 || b >= g->ny, oz = c < 0 || c >= g->nz;
      if ((oy && !pery) || (oz && !perz) || (ox && !perx && !g->open_x))
        return bad(err, "fluid node touches a closed domain edge (make it solid or periodic)");
      if (ox && !perx) continue;  // across the open face
      a = (a + g->nx) % g->nx; b = (b + g->ny) % g->ny; c = (c + g->nz) % g->nz;
      if (!g->solid[a + (int64_t)g->nx * (b + (int64_t)g->ny * c)]) ++nfluid;
    }
    if (g->open_x && (x == 0 || x == g->nx - 1) && nfluid == 0)
      return bad(err, "fluid node on an open face without a fluid neighbour");
    if (rho0) {
      const double r1 = rho0[n], r2 = rho0[N + n];
      if (!std::isfinite(r1) || !std::isfinite(r2) || r1 < 0 || r2 < 0)
        return bad(err, "initial densities must be finite and >= 0");
      if (!(r1 + r2 > 0)) return bad(err, "total initial density must be > 0");
    }
  }
  return true;
}

// Node info words in the pitched layout.
void build_info(const lbm_geometry &g, const Layout &L, std::vector<uint32_t> &info) {
  info.assign((size_t)L.pitch * g.ny * g.nz, kSolid);
  const int q = g.q;
  const bool perx = g.periodic & 1, pery = g.periodic & 2, perz = g.periodic & 4;
  const int x0 = g.porous_x0, x1 = g.porous_x1 > 0 ? g.porous_x1 : g.nx;
  auto solid_at = [&](int a, int b, int c, bool &inside) -> bool {
    inside = true;
    if (a < 0 || a >= g.nx) { if (!perx) { inside = false; return false; } a = (a + g.nx) % g.nx; }
    if (b < 0 || b >= g.ny) { if (!pery) { inside = false; return false; } b = (b + g.ny) % g.ny; }
    if (c < 0 || c >= g.nz) { if (!perz) { inside = false; return false; } c = (c + g.nz) % g.nz; }
    return g.solid[a + (int64_t)g.nx * (b + (int64_t)g.ny * c)] != 0;
  };
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const int64_t n = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
        uint32_t w = 0;
        if (g.solid[n]) {
          w = kSolid;
          for (int i = 1; i < q; ++i) {
            const int *e = evec(q, i);
            bool in;
            const bool s = solid_at(x + e[0], y + e[1], z + e[2], in);
            if (in && !s) w |= 1u << i;
          }
        } else {
          for (int i = 1; i < q; ++i) {
            const int *e = evec(q, i);
            bool in;
            const bool s = solid_at(x - e[0], y - e[1], z - e[2], in);
            if (in && s) w |= 1u << i;
          }
          if (g.open_x && x == 0) w |= kInlet;
          if (g.open_x && x == g.nx - 1) w |= kOutlet;
          if (x >= x0 && x < x1) w |= kWindow;
          if (x == 0 || x == g.nx - 1) {
            // boundary pressure uses face nodes at least 3 nodes from any solid
            bool far = true;
            const int rz = g.nz > 1 ? 2 : 0;
            for (int dz = -rz; dz <= rz && far; ++dz)
              for (int dy = -2; dy <= 2 && far; ++dy)
                for (int dx = -2; dx <= 2 && far; ++dx) {
                  bool in;
                  if (solid_at(x + dx, y + dy, z + dz, in) && in) far = false;
                }
            if (far) w |= kPFace;
          }
        }
        info[(size_t)x + (size_t)L.pitch * (y + (size_t)g.ny * z)] = w;
      }
}

}  // namespace

// ---------------------------------------------------------------------------
struct lbm_batch {
  int32_t k = 0, q = 9, storage = 0, collision = 0, math = 0;
  int32_t strategy = LBM_FUSED, ty = 12;
  bool compact = false;  // compacted layout: only the compact step runs on it
  std::vector<InstDev> h;
  std::vector<Layout> lay;
  std::vector<uint64_t> geom_hash;
  InstDev *d_insts = nullptr;
  int32_t *d_block_inst = nullptr;
  int64_t table_cap = 0;
  int64_t n_blocks = 0;
  double *partials = nullptr;
  double *result = nullptr;
  int obs_blocks = 1;
  hipStream_t stream = nullptr;
  int parity = 0;
  int64_t step = 0;
  bool unstable = false;
  std::string err;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int64_t graph_n = 0;
  int graph_parity = 0;
  // compacted 3D fused step: compact -> dense node keys per instance (host
  // copy, for the edge lists) and whether the carried psi matches the state
  std::vector<std::vector<uint32_t>> ckey_host;
  bool psi_valid = false;
  // retirement: per instance whether it advances, its two own population
  // buffers (a retired instance points both f slots at its current one),
  // the steps it has taken and whether its last observables were non-finite
  std::vector<uint8_t> active;
  std::vector<std::pair<float *, float *>> fown;
  std::vector<int64_t> inst_step;
  std::vector<uint8_t> bad;
};

struct lbm_ctx {
  lbm_batch *b;
};

namespace {

lbm_status fail(lbm_batch *b, lbm_status s, const std::string &msg) {
  if (b) b->err = msg;
  g_err = msg;
  return s;
}

#define HIPCHK(b, expr)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(b, LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

// AUTO's layout for a D2Q9 batch (a single context is a batch of one):
// dense while the two population buffers of all instances fit in the
// 256 MB last-level (Infinity) cache, compacted beyond it.  Measured on
// MI355X: from the cache the dense fused step wins (1024x512: 21.8 against
// 24.4 us), since the compacted pulls put a rank lookup in front of every
// neighbour load; from HBM the compacted layout moves ~40 % fewer bytes and
// its fused step wins (64 instances, 16.4 M nodes: 0.52 against 0.75 ms).
// Instances with an explicit strategy keep it.
constexpr size_t kLastLevelCacheBytes = (size_t)256 << 20;
std::vector<lbm_params> auto_layout(int32_t k, const lbm_geometry *g, const lbm_params *p) {
  std::vector<lbm_params> e(p, p + k);
  if (g[0].q != 9) return e;
  size_t dense = 0;
  for (int i = 0; i < k; ++i) {
    if (p[i].strategy != LBM_AUTO || g[i].q != 9 || !compact_fits(g[i])) return e;
    dense += 2 * make_layout(g[i], p[i]).buf_bytes;
  }
  if (dense <= kLastLevelCacheBytes) return e;
  for (lbm_params &x : e) x.strategy = LBM_COMPACT_FUSED;
  return e;
}

size_t batch_bytes(int32_t k, const lbm_geometry *g, const lbm_params *p, int64_t *n_blocks_out,
                   int *obs_blocks_out) {
  const std::vector<lbm_params> pe = auto_layout(k, g, p);
  p = pe.data();
  size_t bytes = align_up(sizeof(InstDev) * (size_t)k);
  int64_t nb = 0;
  int ob = 1;
  for (int i = 0; i < k; ++i) {
    const Layout L = make_layout(g[i], p[i]);
    nb += std::max(make_tiling(g[i].q, g[i].nx, g[i].ny, g[i].nz, 8).blocks,
                   make_tiling(g[i].q, g[i].nx, g[i].ny, g[i].nz, 8, LBM_COMPACT_FUSED).blocks);
    bytes += L.info_bytes + L.frozen_bytes + L.psi_bytes + 2 * L.buf_bytes;
    if (L.compact) bytes += L.cword_bytes + 2 * L.ckey_bytes + L.cbnd_bytes + L.cedge_bytes;
    InstDev tmp{};
    tmp.nx = g[i].nx; tmp.ny = g[i].ny; tmp.nz = g[i].nz;
    ob = std::max(ob, obs_blocks(tmp));
  }
  bytes += align_up(sizeof(int32_t) * (size_t)nb);
  bytes += align_up(sizeof(double) * kObsFields * (size_t)ob);
  bytes += align_up(sizeof(double) * kObsFields * (size_t)k);
  if (n_blocks_out) *n_blocks_out = nb;
  if (obs_blocks_out) *obs_blocks_out = ob;
  return bytes;
}

// Tilings, block table and descriptors for a step variant; synchronises.
lbm_status apply_plan(lbm_batch *b, int strategy, int ty) {
  if (b->compact != compact_strategy(strategy))
    return fail(b, LBM_EINVAL, "the compact step and the compacted layout go together");
  std::vector<int32_t> table;
  int64_t base = 0;
  for (int i = 0; i < b->k; ++i) {
    InstDev &h = b->h[(size_t)i];
    const Tiling t = make_tiling(b->q, h.nx, h.ny, h.nz, ty, strategy);
    h.tiles_x = t.tiles_x; h.tiles_y = t.tiles_y; h.tiles_z = t.tiles_z;
    h.block_base = (int32_t)base;
    if (!b->active[(size_t)i]) continue;  // retired: no blocks in the table
    for (int64_t j = 0; j < t.blocks; ++j) table.push_back(i);
    base += t.blocks;
  }
  if (base > b->table_cap) return fail(b, LBM_EINVAL, "block table capacity exceeded");
  // compacted 3D fused step: the fluid nodes whose next-step densities the
  // tile march does not complete (outer ring of each tile, end planes of
  // each z chunk), in compact order
  for (int i = 0; i < b->k; ++i) {
    InstDev &h = b->h[(size_t)i];
    h.nedge = 0;
    if (!(b->q == 19 && strategy == LBM_COMPACT_FUSED)) continue;
    std::vector<uint32_t> edge;
    const std::vector<uint32_t> &key = b->ckey_host[(size_t)i];
    const int zlen = (h.nz + h.tiles_z - 1) / h.tiles_z;
    for (size_t c = 0; c < key.size(); ++c) {
      const uint32_t r = key[c] / (uint32_t)h.pitch;
      const int x = (int)(key[c] - r * (uint32_t)h.pitch), y = (int)(r % (uint32_t)h.ny), z = (int)(r / (uint32_t)h.ny);
      const int x0 = x / 64 * 64, y0 = y / kFwdRows * kFwdRows, z0 = z / zlen * zlen;
      const int W = std::min(64, h.nx - x0), H = std::min(kFwdRows, h.ny - y0), z1 = std::min(h.nz, z0 + zlen);
      const bool inner = x - x0 >= 1 && x - x0 <= W - 2 && y - y0 >= 1 && y - y0 <= H - 2 && z > z0 && z < z1 - 1;
      if (!inner) edge.push_back((uint32_t)c);
    }
    h.nedge = (int64_t)edge.size();
    if (!edge.empty())
      HIPCHK(b, hipMemcpyAsync((void *)h.cedge, edge.data(), sizeof(uint32_t) * edge.size(), hipMemcpyHostToDevice,
                               b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));  // the host list dies here
  }
  b->psi_valid = false;
  b->strategy = strategy;
  b->ty = ty;
  b->n_blocks = base;
  if (!table.empty())
    HIPCHK(b, hipMemcpyAsync(b->d_block_inst, table.data(), sizeof(int32_t) * table.size(),
                             hipMemcpyHostToDevice, b->stream));
  HIPCHK(b, hipMemcpyAsync(b->d_insts, b->h.data(), sizeof(InstDev) * b->h.size(), hipMemcpyHostToDevice,
                           b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return LBM_OK;
}

StepLaunch step_launch(const lbm_batch *b, int parity) {
  StepLaunch L;
  L.d_insts = b->d_insts;
  L.h = b->h.data();
  L.block_inst = b->k > 1 ? b->d_block_inst : nullptr;
  L.active = b->active.data();
  L.n_blocks = b->n_blocks;
  L.k = b->k; L.q = b->q; L.collision = b->collision; L.storage = b->storage; L.math = b->math;
  L.strategy = b->strategy; L.ty = b->ty; L.parity = parity;
  return L;
}

lbm_status create_batch(int32_t k, const lbm_geometry *g, const lbm_params *p,
                        const double *const *rho0, void *ws, size_t ws_bytes, void *stream,
                        lbm_batch **out) {
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (k < 1 || !g || !p || !rho0) return fail(nullptr, LBM_EINVAL, "need k >= 1 and non-NULL arrays");
  std::string err;
  for (int i = 0; i < k; ++i) {
    if (!rho0[i]) return fail(nullptr, LBM_EINVAL, "rho_init is NULL");
    if (!validate(&g[i], &p[i], rho0[i], err))
      return fail(nullptr, LBM_EINVAL, (k > 1 ? "instance " + std::to_string(i) + ": " : "") + err);
    if (g[i].q != g[0].q || p[i].storage != p[0].storage || p[i].collision != p[0].collision ||
        p[i].math != p[0].math)
      return fail(nullptr, LBM_EINVAL, "all instances must share q, storage, collision and math");
    if (compact_strategy(resolve_strategy(g[i], p[i])) != compact_strategy(resolve_strategy(g[0], p[0])))
      return fail(nullptr, LBM_EINVAL, "all instances or none must use the compacted layout");
  }
  const std::vector<lbm_params> pe = auto_layout(k, g, p);
  p = pe.data();
  int64_t nb;
  int ob;
  const size_t need = batch_bytes(k, g, p, &nb, &ob);
  if (!ws) return fail(nullptr, LBM_EINVAL, "workspace is NULL");
  if (ws_bytes < need)
    return fail(nullptr, LBM_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(nullptr, LBM_ENOMEM, "workspace must be 256-byte aligned");
  if (nb > 0x7fffffff) return fail(nullptr, LBM_EINVAL, "too many blocks");

  lbm_batch *b = new lbm_batch();
  std::unique_ptr<lbm_batch> owner(b);  // freed on every error return below
  b->k = k;
  b->q = g[0].q;
  b->storage = p[0].storage;
  b->collision = p[0].collision;
  b->math = p[0].math;
  b->stream = reinterpret_cast<hipStream_t>(stream);
  b->n_blocks = nb;
  b->obs_blocks = ob;
  char *cur = reinterpret_cast<char *>(ws);
  auto take = [&](size_t n) { char *r = cur; cur += align_up(n); return r; };
  b->d_insts = reinterpret_cast<InstDev *>(take(sizeof(InstDev) * (size_t)k));
  b->d_block_inst = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)nb));
  b->partials = reinterpret_cast<double *>(take(sizeof(double) * kObsFields * (size_t)ob));
  b->result = reinterpret_cast<double *>(take(sizeof(double) * kObsFields * (size_t)k));

  b->table_cap = nb;
  std::vector<uint32_t> info;
  for (int i = 0; i < k; ++i) {
    const Layout L = make_layout(g[i], p[i]);
    InstDev h{};
    h.info = reinterpret_cast<const uint32_t *>(take(L.info_bytes));
    h.frozen = reinterpret_cast<const float *>(take(L.frozen_bytes));
    h.ivsd0 = L.ivsd0_off ? reinterpret_cast<const float *>(reinterpret_cast<const char *>(h.frozen) + L.ivsd0_off)
                          : nullptr;
    h.psi = reinterpret_cast<float *>(take(L.psi_bytes));
    h.f[0] = reinterpret_cast<float *>(take(L.buf_bytes));
    h.f[1] = reinterpret_cast<float *>(take(L.buf_bytes));
    h.ystride = L.ystride;
    h.zstride = L.zstride;
    h.nx = g[i].nx; h.ny = g[i].ny; h.nz = g[i].nz; h.pitch = L.pitch;
    h.periodic = (int32_t)g[i].periodic; h.open_x = g[i].open_x;
    h.bc_set = p[i].bc_set; h.collision = p[i].collision;
    h.half_shift = p[i].half_force_shift; h.sj_mode = p[i].mrt_sj_mode;
    h.storage = p[i].storage; h.q = g[i].q;
    h.eq26_mode = p[i].eq26_mode;
    h.tau1 = p[i].tau[0]; h.tau2 = p[i].tau[1];
    h.G = p[i].G;
    h.chi1 = 1.0 + p[i].xi; h.chi2 = 1.0 - p[i].xi;
    h.gx = p[i].g[0]; h.gy = p[i].g[1]; h.gz = p[i].g[2];
    h.rho_in1 = p[i].rho_in1; h.rho_out2 = p[i].rho_out2;
    h.rho_in2 = p[i].rho_in2; h.rho_out1 = p[i].rho_out1;
    h.lambda = p[i].lambda; h.s_e = p[i].s_e; h.s_eps = p[i].s_eps;
    // node table
    build_info(g[i], L, info);
    HIPCHK(b, hipMemcpyAsync((void *)h.info, info.data(), sizeof(uint32_t) * info.size(),
                             hipMemcpyHostToDevice, b->stream));
    std::vector<RowWord> cw;
    std::vector<uint32_t> ck, cb;
    if (L.compact) {
      h.compact = 1;
      h.cpitch = L.cpitch;
      h.cword = reinterpret_cast<const RowWord *>(take(L.cword_bytes));
      h.ckey = reinterpret_cast<const uint32_t *>(take(L.ckey_bytes));
      h.cinfo = reinterpret_cast<const uint32_t *>(take(L.ckey_bytes));
      h.cbnd = reinterpret_cast<const uint32_t *>(take(L.cbnd_bytes));
      if (L.cedge_bytes) h.cedge = reinterpret_cast<const uint32_t *>(take(L.cedge_bytes));
      build_compact(g[i], L, info, cw, ck, cb, p[i].tile_rows);
      h.nf = (int64_t)ck.size();
      h.nbnd = (int64_t)cb.size();
      HIPCHK(b, hipMemcpyAsync((void *)h.cword, cw.data(), sizeof(RowWord) * cw.size(), hipMemcpyHostToDevice,
                               b->stream));
      if (!ck.empty()) {
        HIPCHK(b, hipMemcpyAsync((void *)h.ckey, ck.data(), sizeof(uint32_t) * ck.size(), hipMemcpyHostToDevice,
                                 b->stream));
        std::vector<uint32_t> ci(ck.size());
        for (size_t c = 0; c < ck.size(); ++c) ci[c] = info[ck[c]];
        HIPCHK(b, hipMemcpyAsync((void *)h.cinfo, ci.data(), sizeof(uint32_t) * ci.size(), hipMemcpyHostToDevice,
                                 b->stream));
        HIPCHK(b, hipStreamSynchronize(b->stream));  // ci is freed at the end of this block
      }
      if (!cb.empty())
        HIPCHK(b, hipMemcpyAsync((void *)h.cbnd, cb.data(), sizeof(uint32_t) * cb.size(), hipMemcpyHostToDevice,
                                 b->stream));
    }
    b->h.push_back(h);
    b->lay.push_back(L);
    b->active.push_back(1);
    b->fown.emplace_back(h.f[0], h.f[1]);
    b->inst_step.push_back(0);
    b->bad.push_back(0);
    b->ckey_host.push_back(g[i].q == 19 ? ck : std::vector<uint32_t>());
    b->geom_hash.push_back(geometry_hash(g[i]));
    // held (frozen) links: rest equilibria of the initial densities
    const int64_t N = L.n_nodes;
    const int64_t nt = (int64_t)g[i].ny * g[i].nz;
    std::vector<float> frz((size_t)(2 * g[i].q * nt), 0.f);
    for (int64_t t = 0; t < nt; ++t) {
      const int64_t no = (g[i].nx - 1) + (int64_t)g[i].nx * t, ni = (int64_t)g[i].nx * t;
      for (int qi = 0; qi < g[i].q; ++qi) {
        frz[(size_t)(qi * nt + t)] = (float)(weight(g[i].q, qi) * rho0[i][no]);
        frz[(size_t)((g[i].q + qi) * nt + t)] = (float)(weight(g[i].q, qi) * rho0[i][N + ni]);
      }
    }
    HIPCHK(b, hipMemcpyAsync((void *)h.frozen, frz.data(), sizeof(float) * frz.size(),
                             hipMemcpyHostToDevice, b->stream));
    // initial densities staged as float in the psi array (16 bytes per node,
    // always large enough; every step rewrites it before reading), then rest
    // equilibria into buffer 0
    std::vector<float> r0((size_t)(2 * N));
    for (int64_t n = 0; n < 2 * N; ++n) r0[(size_t)n] = (float)rho0[i][n];
    HIPCHK(b, hipMemcpyAsync(h.psi, r0.data(), sizeof(float) * r0.size(), hipMemcpyHostToDevice, b->stream));
    HIPCHK(b, hipMemcpyAsync(b->d_insts + i, &b->h.back(), sizeof(InstDev), hipMemcpyHostToDevice, b->stream));
    HIPCHK(b, launch_init(b->d_insts + i, h, h.psi, 0, b->stream));
    if (h.ivsd0) HIPCHK(b, launch_ivsd_freeze(b->d_insts + i, h, 0, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));  // host staging vectors die here
  }
  // default plan: the split step for D3Q19 (its per-block working set does
  // not fit the L2), the fused step otherwise
  int strategy = resolve_strategy(g[0], p[0]);
  b->compact = compact_strategy(strategy);
  const lbm_status ps = apply_plan(b, strategy, p[0].tile_rows ? p[0].tile_rows : 12);
  if (ps != LBM_OK) return ps;
  *out = owner.release();
  return LBM_OK;
}

// The compacted 3D fused step carries the next step's psi; rebuild it from
// the current state when set-up, a load, new boundary densities, a change
// of step variant or a density read-out staged through it left it stale.
bool carries_psi(const lbm_batch *b) { return b->q == 19 && b->strategy == LBM_COMPACT_FUSED; }

lbm_status ensure_psi(lbm_batch *b) {
  if (!carries_psi(b) || b->psi_valid) return LBM_OK;
  for (int i = 0; i < b->k; ++i)
    if (b->active[(size_t)i]) HIPCHK(b, launch_fwd_rebuild(b->d_insts + i, b->h[i], b->parity, b->stream));
  b->psi_valid = true;
  return LBM_OK;
}

lbm_status batch_step(lbm_batch *b, int64_t n) {
  if (!b) return fail(nullptr, LBM_EINVAL, "NULL handle");
  if (n < 0) return fail(b, LBM_EINVAL, "n must be >= 0");
  if (b->unstable) return fail(b, LBM_EUNSTABLE, "state is unstable (non-finite density)");
  if (n > 0) {
    const lbm_status st = ensure_psi(b);
    if (st != LBM_OK) return st;
  }
  for (int64_t s = 0; s < n; ++s) {
    HIPCHK(b, launch_step(step_launch(b, b->parity), b->stream));
    b->parity ^= 1;
    b->step++;
  }
  for (int i = 0; i < b->k; ++i)
    if (b->active[(size_t)i]) b->inst_step[(size_t)i] += n;
  return LBM_OK;
}

lbm_status batch_step_graph(lbm_batch *b, int64_t n, int64_t reps) {
  if (!b) return fail(nullptr, LBM_EINVAL, "NULL handle");
  if (n <= 0 || (n & 1) || reps < 0) return fail(b, LBM_EINVAL, "n must be even and > 0, reps >= 0");
  if (!b->stream) return fail(b, LBM_ESTATE, "graph capture needs a non-default stream");
  if (b->unstable) return fail(b, LBM_EUNSTABLE, "state is unstable (non-finite density)");
  if (reps > 0) {
    const lbm_status st = ensure_psi(b);
    if (st != LBM_OK) return st;
  }
  if (!b->gexec || b->graph_n != n || b->graph_parity != b->parity) {
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    HIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int par = b->parity;
    for (int64_t s = 0; s < n; ++s) {
      hipError_t e = launch_step(step_launch(b, par), b->stream);
      if (e != hipSuccess) {
        hipGraph_t tmp;
        (void)hipStreamEndCapture(b->stream, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        return fail(b, LBM_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
      }
      par ^= 1;
    }
    HIPCHK(b, hipStreamEndCapture(b->stream, &b->graph));
    HIPCHK(b, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    b->graph_n = n;
    b->graph_parity = b->parity;
  }
  for (int64_t r = 0; r < reps; ++r) {
    HIPCHK(b, hipGraphLaunch(b->gexec, b->stream));
    b->step += n;
    for (int i = 0; i < b->k; ++i)
      if (b->active[(size_t)i]) b->inst_step[(size_t)i] += n;
  }
  return LBM_OK;
}

void fill_obs(const lbm_batch *b, int i, const double *r, lbm_obs *o) {
  std::memset(o, 0, sizeof(*o));
  o->step = b->inst_step[(size_t)i];
  o->mass[0] = r[0];
  o->mass[1] = r[1];
  o->n_fluid = r[2];
  o->n_window = r[3];
  o->sw_count = r[4];
  o->sum_rho_w = r[5];
  o->sum_rho = r[6];
  o->s_w = r[3] > 0 ? r[4] / r[3] : 0.0;
  o->s_w_weighted = r[6] > 0 ? r[5] / r[6] : 0.0;
  o->n_in = r[8];
  o->n_out = r[10];
  o->p_in = r[8] > 0 ? r[7] / r[8] : 0.0;
  o->p_out = r[10] > 0 ? r[9] / r[10] : 0.0;
  o->pc = o->p_in - o->p_out;
  o->flags = (int32_t)r[14];
  const double m = r[0] + r[1];
  for (int d = 0; d < 3; ++d) o->stag[d] = m > 0 ? r[11 + d] / m : 0.0;
}

lbm_status batch_observables(lbm_batch *b, lbm_obs *out) {
  if (!b || !out) return fail(b, LBM_EINVAL, "NULL argument");
  for (int i = 0; i < b->k; ++i)
    HIPCHK(b, launch_observables(b->d_insts + i, b->h[i], b->parity, b->partials, obs_blocks(b->h[i]),
                                 b->result + (size_t)kObsFields * i, b->stream));
  std::vector<double> r((size_t)kObsFields * b->k);
  HIPCHK(b, hipMemcpyAsync(r.data(), b->result, sizeof(double) * r.size(), hipMemcpyDeviceToHost, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  bool bad_state = false;
  for (int i = 0; i < b->k; ++i) {
    fill_obs(b, i, r.data() + (size_t)kObsFields * i, out + i);
    // a non-finite density stops the batch unless its instance is retired;
    // a negative density (bit 1) is only reported
    b->bad[(size_t)i] = (out[i].flags & 1) ? 1 : 0;
    if (b->bad[(size_t)i] && b->active[(size_t)i]) bad_state = true;
  }
  if (bad_state) {
    b->unstable = true;
    return fail(b, LBM_EUNSTABLE, "non-finite density");
  }
  return LBM_OK;
}

lbm_status batch_density(lbm_batch *b, int32_t i, float *dst, int32_t dst_is_device) {
  if (!b || !dst) return fail(b, LBM_EINVAL, "NULL argument");
  if (i < 0 || i >= b->k) return fail(b, LBM_EINVAL, "instance index out of range");
  const InstDev &h = b->h[(size_t)i];
  const int64_t N = (int64_t)h.nx * h.ny * h.nz;
  if (dst_is_device) {
    HIPCHK(b, launch_density(b->d_insts + i, h, b->parity, dst, b->stream));
    return LBM_OK;
  }
  // stage in the psi array: 16 bytes per node, so always large enough (the
  // compacted population buffers may hold fewer than 2N floats), and every
  // step rewrites it before reading it
  float *stage = h.psi;
  b->psi_valid = false;
  HIPCHK(b, launch_density(b->d_insts + i, h, b->parity, stage, b->stream));
  HIPCHK(b, hipMemcpyAsync(dst, stage, sizeof(float) * 2 * (size_t)N, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  return LBM_OK;
}

// Checkpoint blob: header, the boundary densities, the held (Eq. 26/27)
// links, the current population buffer, and (compacted 3D fused step) the
// carried psi.  The header records the layout and the geometry, and lbm_load
// restores a blob only onto a context with the same ones.
struct CkptHeader {
  char magic[8];
  int32_t version, k, q, storage;
  int32_t parity, compact;
  int32_t nx, ny, nz, pitch;
  int32_t cpitch, pad;
  int64_t step;
  uint64_t buf_bytes, frozen_bytes, geom_hash;
  double rho_in1, rho_out2;
  uint64_t psi_bytes;  // 0, or the carried psi array (dense float pairs)
};
constexpr int32_t kCkptVersion = 5;

size_t carried_psi_bytes(const InstDev &h) { return (size_t)h.pitch * h.ny * h.nz * 2 * sizeof(float); }
size_t ckpt_bytes(const Layout &L, size_t psi_bytes) {
  return sizeof(CkptHeader) + L.frozen_bytes + L.buf_bytes + psi_bytes;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t lbm_workspace_bytes(const lbm_geometry *geom, const lbm_params *params) {
  std::string err;
  if (!geom || !params) return 0;
  if (!validate(geom, params, nullptr, err)) return 0;
  return batch_bytes(1, geom, params, nullptr, nullptr);
}

lbm_status lbm_create(const lbm_geometry *geom, const lbm_params *params, const double *rho_init,
                      void *workspace, size_t ws_bytes, void *hip_stream, lbm_ctx **out) {
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  const double *r[1] = {rho_init};
  lbm_batch *b = nullptr;
  lbm_status s = create_batch(1, geom, params, r, workspace, ws_bytes, hip_stream, &b);
  if (s != LBM_OK) return s;
  *out = new lbm_ctx{b};
  return LBM_OK;
}

lbm_status lbm_set_bc(lbm_ctx *ctx, double rho_in1, double rho_out2) {
  if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL handle");
  lbm_batch *b = ctx->b;
  if (!std::isfinite(rho_in1) || !std::isfinite(rho_out2) || rho_in1 <= 0 || rho_out2 <= 0)
    return fail(b, LBM_EINVAL, "boundary densities must be finite and > 0");
  b->h[0].rho_in1 = rho_in1;
  b->h[0].rho_out2 = rho_out2;
  b->psi_valid = false;  // the carried inlet/outlet densities follow the old values
  HIPCHK(b, hipMemcpyAsync(b->d_insts, &b->h[0], sizeof(InstDev), hipMemcpyHostToDevice, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *ctx, int64_t n) {
  if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL handle");
  return batch_step(ctx->b, n);
}

lbm_status lbm_step_graph(lbm_ctx *ctx, int64_t n, int64_t reps) {
  if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL handle");
  return batch_step_graph(ctx->b, n, reps);
}

lbm_status lbm_observables(lbm_ctx *ctx, lbm_obs *out) {
  if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL handle");
  return batch_observables(ctx->b, out);
}

lbm_status lbm_get_density(lbm_ctx *ctx, float *dst, int32_t dst_is_device) {
  if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL handle");
  return batch_density(ctx->b, 0, dst, dst_is_device);
}

lbm_status lbm_save(lbm_ctx *ctx, void *host_blob, size_t *bytes) {
  if (!ctx || !bytes) return fail(nullptr, LBM_EINVAL, "NULL argument");
  lbm_batch *b = ctx->b;
  const Layout &L = b->lay[0];
  const size_t pb = carries_psi(b) ? carried_psi_bytes(b->h[0]) : 0;
  const size_t need = ckpt_bytes(L, pb);
  if (!host_blob) { *bytes = need; return LBM_OK; }
  if (*bytes < need) return fail(b, LBM_EINVAL, "checkpoint buffer too small");
  if (pb) {
    const lbm_status st = ensure_psi(b);
    if (st != LBM_OK) return st;
  }
  const InstDev &h = b->h[0];
  CkptHeader hd{};
  std::memcpy(hd.magic, "LBMCKPT", 8);
  hd.version = kCkptVersion; hd.k = 1; hd.q = b->q; hd.storage = b->storage;
  hd.parity = b->parity; hd.compact = L.compact ? 1 : 0;
  hd.nx = h.nx; hd.ny = h.ny; hd.nz = h.nz; hd.pitch = L.pitch; hd.cpitch = L.cpitch;
  hd.step = b->step;
  hd.buf_bytes = L.buf_bytes; hd.frozen_bytes = L.frozen_bytes; hd.geom_hash = b->geom_hash[0];
  hd.rho_in1 = h.rho_in1; hd.rho_out2 = h.rho_out2;
  hd.psi_bytes = pb;
  char *p = reinterpret_cast<char *>(host_blob);
  std::memcpy(p, &hd, sizeof(hd));
  HIPCHK(b, hipMemcpyAsync(p + sizeof(hd), h.frozen, L.frozen_bytes, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(b, hipMemcpyAsync(p + sizeof(hd) + L.frozen_bytes, h.f[b->parity], L.buf_bytes, hipMemcpyDeviceToHost,
                           b->stream));
  if (pb)
    HIPCHK(b, hipMemcpyAsync(p + sizeof(hd) + L.frozen_bytes + L.buf_bytes,
                             reinterpret_cast<const char *>(h.psi) + (size_t)b->parity * pb, pb,
                             hipMemcpyDeviceToHost, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  *bytes = need;
  return LBM_OK;
}

lbm_status lbm_load(lbm_ctx *ctx, const void *host_blob, size_t bytes) {
  if (!ctx || !host_blob) return fail(nullptr, LBM_EINVAL, "NULL argument");
  lbm_batch *b = ctx->b;
  const Layout &L = b->lay[0];
  if (bytes < sizeof(CkptHeader)) return fail(b, LBM_EINVAL, "checkpoint too small");
  CkptHeader hd;
  std::memcpy(&hd, host_blob, sizeof(hd));
  if (hd.psi_bytes != 0 && hd.psi_bytes != carried_psi_bytes(b->h[0]))
    return fail(b, LBM_EINVAL, "corrupt checkpoint (carried psi size)");
  const size_t need = ckpt_bytes(L, (size_t)hd.psi_bytes);
  const InstDev &cur = b->h[0];
  if (std::memcmp(hd.magic, "LBMCKPT", 8) || hd.version != kCkptVersion || hd.k != 1)
    return fail(b, LBM_EINVAL, "not a checkpoint of this library version");
  if (bytes != need || hd.q != b->q || hd.storage != b->storage || hd.compact != (L.compact ? 1 : 0) ||
      hd.nx != cur.nx || hd.ny != cur.ny || hd.nz != cur.nz || hd.pitch != L.pitch || hd.cpitch != L.cpitch ||
      hd.buf_bytes != L.buf_bytes || hd.frozen_bytes != L.frozen_bytes || hd.geom_hash != b->geom_hash[0])
    return fail(b, LBM_EINVAL, "checkpoint does not match this context (lattice, storage, layout or geometry)");
  if (hd.parity != 0 && hd.parity != 1) return fail(b, LBM_EINVAL, "corrupt checkpoint (buffer parity)");
  if (hd.step < 0 || !std::isfinite(hd.rho_in1) || !std::isfinite(hd.rho_out2))
    return fail(b, LBM_EINVAL, "corrupt checkpoint (step or boundary densities)");
  const char *p = reinterpret_cast<const char *>(host_blob);
  b->parity = hd.parity;
  b->step = hd.step;
  b->inst_step[0] = hd.step;
  b->bad[0] = 0;
  b->h[0].rho_in1 = hd.rho_in1;
  b->h[0].rho_out2 = hd.rho_out2;
  HIPCHK(b, hipMemcpyAsync((void *)b->h[0].frozen, p + sizeof(hd), L.frozen_bytes, hipMemcpyHostToDevice,
                           b->stream));
  HIPCHK(b, hipMemcpyAsync(b->h[0].f[b->parity], p + sizeof(hd) + L.frozen_bytes, L.buf_bytes,
                           hipMemcpyHostToDevice, b->stream));
  // a carried psi is restored only for the step that carries it; otherwise
  // it is rebuilt from the state before the next step
  b->psi_valid = hd.psi_bytes != 0 && carries_psi(b);
  if (b->psi_valid)
    HIPCHK(b, hipMemcpyAsync(reinterpret_cast<char *>(b->h[0].psi) + (size_t)b->parity * hd.psi_bytes,
                             p + sizeof(hd) + L.frozen_bytes + L.buf_bytes, hd.psi_bytes, hipMemcpyHostToDevice,
                             b->stream));
  HIPCHK(b, hipMemcpyAsync(b->d_insts, &b->h[0], sizeof(InstDev), hipMemcpyHostToDevice, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  b->unstable = false;
  return LBM_OK;
}

lbm_status lbm_debug_poke(lbm_ctx *ctx, int32_t x, int32_t y, int32_t z, int32_t s, int32_t i, float value) {
  if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL handle");
  lbm_batch *b = ctx->b;
  const InstDev &h = b->h[0];
  if (x < 0 || x >= h.nx || y < 0 || y >= h.ny || z < 0 || z >= h.nz)
    return fail(b, LBM_EINVAL, "node outside the grid");
  if (s < 0 || s > 1 || i < 0 || i >= h.q) return fail(b, LBM_EINVAL, "component must be 0 or 1, link in [0, q)");
  int32_t *status = reinterpret_cast<int32_t *>(b->result);
  HIPCHK(b, launch_poke(b->d_insts, h, b->parity, x, y, z, s, i, value, status, b->stream));
  int32_t st = -1;
  HIPCHK(b, hipMemcpyAsync(&st, status, sizeof st, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  if (st != 0) return fail(b, LBM_EINVAL, "node is solid");
  b->psi_valid = false;  // the carried psi followed the old value
  return LBM_OK;
}

lbm_status lbm_init_from_saturation(lbm_ctx *ctx, const float *sat, int32_t sat_is_device, double threshold,
                                    double rho_major, double rho_minor) {
  if (!ctx || !sat) return fail(nullptr, LBM_EINVAL, "NULL argument");
  lbm_batch *b = ctx->b;
  if (!std::isfinite(threshold) || !std::isfinite(rho_major) || !std::isfinite(rho_minor) || rho_major < 0 ||
      rho_minor < 0 || !(rho_major + rho_minor > 0))
    return fail(b, LBM_EINVAL, "densities must be finite and >= 0 with a positive sum");
  const InstDev &h = b->h[0];
  const float *src = sat;
  if (!sat_is_device) {
    // stage in the psi buffer (16 bytes per node); the carried psi is rebuilt
    float *stage = h.psi;
    HIPCHK(b, hipMemcpyAsync(stage, sat, sizeof(float) * (size_t)h.nx * h.ny * h.nz, hipMemcpyHostToDevice,
                             b->stream));
    src = stage;
  }
  HIPCHK(b, launch_init_sat(b->d_insts, h, src, (float)threshold, (float)rho_major, (float)rho_minor, b->parity,
                            b->stream));
  if (h.ivsd0) HIPCHK(b, launch_ivsd_freeze(b->d_insts, h, b->parity, b->stream));
  if (!sat_is_device) HIPCHK(b, hipStreamSynchronize(b->stream));
  b->psi_valid = false;
  b->unstable = false;
  b->step = 0;
  b->inst_step[0] = 0;
  b->bad[0] = 0;
  return LBM_OK;
}

int64_t lbm_get_step(const lbm_ctx *ctx) { return ctx ? ctx->b->step : -1; }

lbm_status lbm_destroy(lbm_ctx *ctx) {
  if (!ctx) return LBM_OK;
  lbm_batch_destroy(ctx->b);
  delete ctx;
  return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *ctx) {
  if (ctx && ctx->b) return ctx->b->err.c_str();
  return g_err.c_str();
}

lbm_status lbm_kernel_info(const lbm_ctx *ctx, char *name, size_t name_len, int64_t *grid_blocks,
                           int32_t *block_threads) {
  if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL handle");
  return lbm_batch_kernel_info(ctx->b, name, name_len, grid_blocks, block_threads);
}

lbm_status lbm_batch_kernel_info(const lbm_batch *b, char *name, size_t name_len, int64_t *grid_blocks,
                                 int32_t *block_threads) {
  if (!b) return fail(nullptr, LBM_EINVAL, "NULL handle");
  if (name && name_len)
    std::snprintf(name, name_len, "%s", step_kernel_name(b->q, b->collision, b->storage, b->math, b->strategy, b->ty));
  if (grid_blocks) {
    if (b->strategy == LBM_SPLIT) {  // one launch per instance: the largest grid
      int64_t g = 0;
      for (const InstDev &h : b->h) g = std::max(g, ((int64_t)((h.nx + 63) / 64) * h.ny * h.nz + 3) / 4);
      *grid_blocks = g;
    } else if (b->strategy == LBM_COMPACT) {
      int64_t g = 0;
      for (const InstDev &h : b->h) g = std::max(g, (h.nf + kCompactThreads - 1) / kCompactThreads);
      *grid_blocks = g;
    } else {
      *grid_blocks = b->n_blocks;
    }
  }
  if (block_threads) *block_threads = b->strategy == LBM_COMPACT ? kCompactThreads : 256;
  return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx *ctx, int64_t steps, char *report, size_t report_len) {
  if (!ctx) return fail(nullptr, LBM_EINVAL, "NULL handle");
  return lbm_batch_autotune(ctx->b, steps, report, report_len);
}

lbm_status lbm_batch_autotune(lbm_batch *b, int64_t steps, char *report, size_t report_len) {
  if (!b) return fail(nullptr, LBM_EINVAL, "NULL handle");
  if (steps < 2 || (steps & 1)) return fail(b, LBM_EINVAL, "steps must be even and >= 2");
  struct Cand { int strategy, ty; };
  std::vector<Cand> cands;
  if (b->compact) {
    cands.push_back({LBM_COMPACT, 12});
    if (b->q == 9)
      for (int ty : {8, 12, 16}) cands.push_back({LBM_COMPACT_FUSED, ty});
    else if (b->storage == LBM_STORE_F32)
      cands.push_back({LBM_COMPACT_FUSED, 12});
  } else {
    if (b->q == 9) {
      for (int ty : {8, 12, 16}) cands.push_back({LBM_FUSED, ty});
      bool fits = true;
      for (const InstDev &h : b->h) fits = fits && list_fits(h.nx);
      if (fits)
        for (int ty : {8, 12, 16}) cands.push_back({LBM_FUSED_LIST, ty});
    } else {
      cands.push_back({LBM_FUSED, 12});
    }
    cands.push_back({LBM_SPLIT, 12});
  }
  hipEvent_t e0, e1;
  HIPCHK(b, hipEventCreate(&e0));
  HIPCHK(b, hipEventCreate(&e1));
  // two passes over the variants, the better time of each counting: a single
  // short trial right after a switch of variant can land several percent off
  std::vector<float> ms_best(cands.size(), 1e30f);
  for (int pass = 0; pass < 2; ++pass)
    for (size_t ci = 0; ci < cands.size(); ++ci) {
      const Cand &c = cands[ci];
      lbm_status st = apply_plan(b, c.strategy, c.ty);
      if (st != LBM_OK) return st;
      st = batch_step(b, 2);  // warm-up
      if (st != LBM_OK) return st;
      HIPCHK(b, hipEventRecord(e0, b->stream));
      st = batch_step(b, steps);
      if (st != LBM_OK) return st;
      HIPCHK(b, hipEventRecord(e1, b->stream));
      HIPCHK(b, hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(b, hipEventElapsedTime(&ms, e0, e1));
      ms_best[ci] = std::min(ms_best[ci], ms / (float)steps);
    }
  std::string rep;
  float best = 1e30f;
  Cand bestc = cands[0];
  for (size_t ci = 0; ci < cands.size(); ++ci) {
    const Cand &c = cands[ci];
    char line[128];
    std::snprintf(line, sizeof line, "%s %.5f ms/step\n",
                  step_kernel_name(b->q, b->collision, b->storage, b->math, c.strategy, c.ty), ms_best[ci]);
    rep += line;
    if (ms_best[ci] < best) { best = ms_best[ci]; bestc = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  lbm_status st = apply_plan(b, bestc.strategy, bestc.ty);
  if (st != LBM_OK) return st;
  if (report && report_len) std::snprintf(report, report_len, "%s", rep.c_str());
  return LBM_OK;
}

size_t lbm_batch_workspace_bytes(int32_t k, const lbm_geometry *geoms, const lbm_params *params) {
  if (k < 1 || !geoms || !params) return 0;
  std::string err;
  for (int i = 0; i < k; ++i)
    if (!validate(&geoms[i], &params[i], nullptr, err)) return 0;
  return batch_bytes(k, geoms, params, nullptr, nullptr);
}

lbm_status lbm_batch_create(int32_t k, const lbm_geometry *geoms, const lbm_params *params,
                            const double *const *rho_inits, void *workspace, size_t ws_bytes,
                            void *hip_stream, lbm_batch **out) {
  return create_batch(k, geoms, params, rho_inits, workspace, ws_bytes, hip_stream, out);
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t n) { return batch_step(b, n); }
lbm_status lbm_batch_step_graph(lbm_batch *b, int64_t n, int64_t reps) { return batch_step_graph(b, n, reps); }
lbm_status lbm_batch_observables(lbm_batch *b, lbm_obs *out) { return batch_observables(b, out); }

// Retire or re-admit instances.  A retired instance keeps its state in the
// buffer it was left in: both f slots point there, so every read (density,
// observables) finds it whatever the batch parity; re-admission gives it its
// other buffer back as the next step's destination.
lbm_status lbm_batch_set_active(lbm_batch *b, const int32_t *active) {
  if (!b) return fail(nullptr, LBM_EINVAL, "NULL handle");
  if (!active) return fail(b, LBM_EINVAL, "active is NULL");
  bool changed = false;
  for (int i = 0; i < b->k; ++i) {
    const uint8_t want = active[i] ? 1 : 0;
    if (want == b->active[(size_t)i]) continue;
    changed = true;
    InstDev &h = b->h[(size_t)i];
    const std::pair<float *, float *> &own = b->fown[(size_t)i];
    float *cur = h.f[b->parity];
    if (!want) {
      h.f[0] = h.f[1] = cur;
    } else {
      h.f[b->parity] = cur;
      h.f[b->parity ^ 1] = cur == own.first ? own.second : own.first;
    }
    b->active[(size_t)i] = want;
  }
  if (!changed) return LBM_OK;
  b->unstable = false;
  for (int i = 0; i < b->k; ++i)
    if (b->active[(size_t)i] && b->bad[(size_t)i]) b->unstable = true;
  // new block table and descriptors; drops the captured graph and the carried psi
  return apply_plan(b, b->strategy, b->ty);
}
lbm_status lbm_batch_get_density(lbm_batch *b, int32_t k, float *dst, int32_t dst_is_device) {
  return batch_density(b, k, dst, dst_is_device);
}

lbm_status lbm_batch_destroy(lbm_batch *b) {
  if (!b) return LBM_OK;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
  return LBM_OK;
}

const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : g_err.c_str(); }

}  // extern "C"
