// Internal declarations of the gfx950 overset grid-assembly library.
// Device-side grid table, context layout and the launchers each kernel file
// provides. Nothing here is part of the C ABI (see include/overset.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "overset.h"

namespace ov {

constexpr int kMaxGrids = OV_MAX_GRIDS;
constexpr uint8_t kHole = OV_STATE_HOLE;
constexpr uint8_t kFringe = OV_STATE_FRINGE;

// Containment and Newton constants: a cell contains a point iff its
// natural coordinates lie in [-kSTol, 1 + kSTol]^3; Newton stops once its
// last step is at most kNewtonTol (FP64).
constexpr double kSTol = 1e-12;
constexpr double kNewtonTol = 1e-12;
constexpr int kNewtonMaxIt = 50;
constexpr double kDetMin = 1e-300;

// Fringe-marking tile (nodes along i, j, k) and the widest buffer supported.
// The hole cut culls per sub-tile (kSubI nodes along i).
constexpr int kTileI = 64, kTileJ = 8, kTileK = 8;
constexpr int kSubI = 16, kSubPerTile = kTileI / kSubI;
// sub-tiles per mask chunk (one per thread of a 256-thread block)
constexpr int kMaskChunk = 256;
constexpr int kMaxNf = 3;
// Compaction chunk: 256 threads x 16 flag bytes; 64 chunks form a superchunk.
constexpr int kCompactThreads = 256;
constexpr int kCompactChunk = kCompactThreads * 16;
constexpr int kSuperChunk = 64;
// Front-half scratch slots: the hole cut and the fringe pass of one step use
// one slot; up to kSlots steps can be between the two at once.
constexpr int kSlots = 3;
constexpr int kSuperSlots = 8;  // count slots per superchunk (spreads the atomics)
constexpr long long kFusedScanMax = 4096;  // superchunks whose offsets one block forms in LDS

// One grid as the kernels see it.
struct GridDev {
  int ni, nj, nk, per;
  int nci, ncj, nck, blank_kind;
  long long node_off, nnodes, ncells;
  double inv_nci, inv_plane;  // 1 / nci and 1 / (nci ncj), rounded: cell decomposition without division
  const double* X;
  const double* Y;
  const double* Z;
  const float* Xf;  // FP32 shadows (mixed precision), else null
  const float* Yf;
  const float* Zf;
  const double4* P;  // (x, y, z, 0) per node: the donor search's gather layout
  // mixed precision: (x, y, z, 0) per node in FP32 as offsets from `anchor`
  // (the centre of the box of the grid's nodes), the FP32 walk's corners;
  // every component's rounding is at most pf_err
  const float4* PF;
  double anchor[3];
  double pf_err;
  double blank_prm[8];
  double cull_r2;  // body-frame sphere about the origin enclosing the blank region, squared
  int outer[6];
  int has_outer;
  int tiles_i, tiles_j, tiles_k;
  long long tile_off;  // first fringe tile of this grid
  // control cells: uniform bins over the body-frame box of the grid's nodes
  double blo[3], bhi[3], binv[3];
  int nb[3];
  // polar ends: bit 2a (low end) and bit 2a + 1 (high end) of axis a set
  // where that face collapses onto lines along the one periodic axis (the
  // axis of a grid of revolution; the cells there are wedges round it)
  int pole;
  const long long* bstart;  // [nbins + 1]
  const int* bcells;        // candidate donor cells, bin after bin (ascending in each bin)
  const int* brep;          // walk seed of each bin (listed cell nearest its centre), -1 if empty
  // second level: a bin listing more than kSplitList cells is split into
  // kSubBins^3 sub-bins with (ascending) lists of their own
  const int* bsub;          // per bin: its first sub-bin, or -1 (null: no bin is split)
  const long long* sstart;  // [nsub + 1]
  const int* scells;
  // OV_BLANK_MESH: the closed surface triangulation (9 doubles per triangle,
  // body frame), its triangles binned by their (y, z) box over a uniform
  // 2-D grid of the surface's (y, z) box (a ray along +x meets only the
  // triangles of its bin)
  const double* mtri;  // per bin its triangles, contiguous, oriented (see mesh_parity)
  const int* mstart;   // [mn[0] * mn[1] + 1], in triangles
  double mbox[6];     // axis-aligned box of the surface: lo x, y, z, hi x, y, z
  double minv[2];     // bins per unit length along y and z
  int mn[2];          // bins along y and z
  // voxels over the box: 0 outside, 1 inside (no triangle's padded box
  // meets the voxel; the status of its centre), 2 the surface may pass
  const uint8_t* mvox;
  double mvinv[3];  // voxels per unit length along x, y, z
  int mvn[3];       // voxels along x, y, z
  int mpad_;
};

struct GridHost {
  GridDev d{};
  // library-owned device buffers of this grid
  float* xf = nullptr;
  float* yf = nullptr;
  float* zf = nullptr;
  double4* p = nullptr;
  float4* pf = nullptr;
  long long* bstart = nullptr;
  int* bcells = nullptr;
  int* brep = nullptr;
  int* bsub = nullptr;
  long long* sstart = nullptr;
  int* scells = nullptr;
  std::vector<double> mesh;  // OV_BLANK_MESH triangles (host copy until finalize)
  double* mtri = nullptr;
  int* mstart = nullptr;
  uint8_t* mvox = nullptr;
};

}  // namespace ov

struct ov_ctx {
  int device = 0;
  int precision = OV_FP64;
  int num_cus = 256;
  bool finalized = false;
  std::vector<ov::GridHost> grids;
  std::vector<long long> node_off{0};
  long long total_tiles = 0;
  long long sub_perm = 1;  // multiplier prime to the sub-tile count: the hole cut's visiting order
  ov::GridDev* d_grids = nullptr;
  int32_t* d_status = nullptr;
  // OV_STAT_* counters (accumulate until ov_stats_fetch), spread over
  // kStatSlots slots of kStatStride words: a workgroup adds to the slot of
  // its index, so that the per-workgroup additions of one launch do not all
  // queue on one address
  unsigned long long* d_stats = nullptr;
  // per node, one 8-byte warm-start record: bits 0-31 the donor cell of its
  // last query, bits 32-39 the donor grid (255: none), bits 40-47 the low
  // byte of the stamp of the step that wrote it (one load and one store per
  // query instead of three of each)
  unsigned long long* d_warm = nullptr;
  double4* d_tile_sphere = nullptr;  // per sub-tile: body-frame bounding sphere (centre, radius; -inf if empty)
  int4* d_tile_info = nullptr;       // per node tile: (grid, ti, tj, tk)
  // The flags every step starts from (field everywhere, fringe on the fixed
  // outer-boundary layers), laid out like the flag array; only the ranges
  // of grids with outer layers are kept (others are all zero). Consecutive
  // grids of one kind form a fill range: 4 values per range (start, end,
  // whole 16-byte words before it, kind 0 = zeros / 1 = copy of the base).
  uint8_t* d_base_flags = nullptr;
  long long* d_fill_ranges = nullptr;
  int n_fill_ranges = 0;
  long long fill_words = 0;
  // Front-half scratch, written and read in stream order by the hole cut,
  // the fringe pass and the compaction. Each hole cut starts a new stamp; a
  // tile or chunk is on this step's list when its entry equals the stamp, so
  // nothing needs clearing between steps.
  unsigned int* d_stamp = nullptr;            // [0] (unused), [1 + slot] stamp of scratch slot `slot`,
                                              // [1 + kSlots] counter of the C-ABI fringe call's own lists
  unsigned int* d_tile_hole = nullptr;        // per slot and tile: the stamp of the slot's step if the tile holds a hole
  // the culled hole cut's candidate lookup (OV_OPT_HOLECUT_LIST): per slot,
  // the blank regions that may reach each sub-tile, computed by the step's
  // start kernel, and the number of sub-tiles with any in each mask chunk
  unsigned long long* d_sub_mask = nullptr;   // [kSlots * nsub]
  int32_t* d_mask_counts = nullptr;           // [kSlots * nmask_chunks]
  long long nmask_chunks = 0;
  unsigned int* d_tile_near = nullptr;        // [slot][tile]: stamp if on the slot's near list
  unsigned int hole_stamp = 0;                // the last stamp numbered on the host (by-step executors)
  int4* d_near_list = nullptr;                // per slot: tiles that may hold buffer nodes (a hole within kMaxNf)
  int32_t* d_near_count = nullptr;            // per slot
  uint8_t* d_chunk_static = nullptr;          // per chunk: holds outer-boundary query nodes
  unsigned int* d_chunk_stamp = nullptr;      // per chunk: stamp if on this step's chunk list
  int32_t* d_chunk_list = nullptr;            // chunks that may hold query nodes: the static ones, then this step's
  int32_t* d_chunk_list_count = nullptr;      // per slot: length of this step's part
  long long n_static_chunks = 0;
  unsigned long long* d_chunk_counts = nullptr;  // per chunk: stamp << 32 | query count (listed chunks)
  int32_t* d_super_counts = nullptr;             // per slot, per 64 chunks, kSuperSlots partial counts
  long long* d_super_offsets = nullptr;          // per 64 chunks: first query position; last entry the total
  long long nchunks = 0, nsuper = 0;
  // options
  int warm = 1;
  int max_walk = 16;
  int search_block = 64;
  int interp_block = 256;
  int holecut_block = 512;
  int holecut_npt = 2;  // 16-byte coordinate vectors per lane per chunk
  int persist = 0;
  int cull = 1;  // hole cut: skip coordinate reads of tiles no blank region can reach
  int holecut_npl = 16;  // candidate nodes per lane in the culled hole cut: 16 (wavefront per sub-tile) or 4 (block)
  int holecut_list = 0;  // culled hole cut: candidates ranked from the start kernel's masks, one per block
  int back_fused = 1;    // step executors: transform, search and interpolation in one kernel
  int back_blocks_per_cu = 8;  // persistent blocks of that kernel per compute unit
  int back_block = 256;        // its threads per block (64, 128 or 256)
  int back_queue = 0;          // its blocks take query chunks from an atomic head (executors)
  int back_xcd = 0;            // runs of this many consecutive chunks go to one XCD (0: launch order)
  int field_layout = 0;        // 0: four blocks u, v, w, p; 1: interleaved per node
  int frame_velocity = 0;      // executors: interpolated velocities in the receiver's frame
  bool has_mesh = false;       // some grid's blank region is a triangulation
  void* static_scratch = nullptr;  // this device's copy of the no-allocation call's static array
  std::string err;
};

namespace ov {

int fail(ov_ctx* ctx, int code, const char* fmt, ...);
int hip_fail(ov_ctx* ctx, hipError_t e, const char* what);
long long grid_size_for(const ov_ctx* ctx, long long items, int block);

// launchers (kernel files)
// slot: which front-half scratch slot (0..kSlots-1) the step uses (the hole
// cut and the fringe/compaction of one step must use the same slot)
// gen: which of the slot's two near lists the step writes (and the fringe
// pass reads); reset: instead of writing every flag, return only the tiles
// on the slot's other near list (the previous step of this slot and flags
// buffer) to their base flags, for callers whose flags buffer holds exactly
// that step's result (the step executors). stamp: 0 numbers the step on the
// device (the context's step counter, advanced by the step's first kernel;
// also under graph capture, where every replay takes the next number);
// otherwise the step's stamp, numbered by the caller in issue order
// (next_hole_stamp), which raises the device counter to it.
hipError_t launch_holecut(ov_ctx* ctx, const double* poses, uint8_t* flags, hipStream_t s, int slot = 0, int gen = 0,
                          bool reset = false, unsigned int stamp = 0u);

// Stamps: 0 marks "never listed"; the high bit keeps the C ABI's fringe
// call's own stamps apart from the hole cut's; the wrap goes on to 2, so that
// the parity of consecutive stamps alternates (the back half picks its queue
// counters by it).
constexpr unsigned int kStampHigh = 0x80000000u;
__host__ __device__ __forceinline__ unsigned int stamp_after(unsigned int v) {
  v = (v + 1u) & ~kStampHigh;
  return v == 0u ? 2u : v;
}
// The scratch of one fringe pass and compaction: the near-tile list, the
// chunk list and the compaction's per-chunk and per-superchunk counts. It
// lives in the context's slots, or (the no-allocation fringe call) in the
// library's static device array.
struct FrontScratch {
  unsigned int* counter;             // step counter: a new stamp is its next value
  unsigned int* stamp;               // this pass's stamp
  int4* near_list;                   // [total_tiles]
  int32_t* near_count;
  unsigned int* tile_near;           // [total_tiles]: stamp if on the near list
  unsigned int* chunk_stamp;         // [nchunks]: stamp if on the chunk list
  int32_t* chunk_list;               // [nchunks]: the static chunks, then this pass's
  int32_t* chunk_list_count;         // length of this pass's part
  unsigned long long* chunk_counts;  // [nchunks]: stamp << 32 | query count
  int32_t* super_counts;             // [kSuperSlots * nsuper]
  long long* super_offsets;          // [nsuper + 1]
};
// Device address of this device's copy of the static scratch array of the
// no-allocation fringe call (looked up once per device; `device` current).
hipError_t static_scratch_address(int device, void** out);
// The context's scratch of slot `slot` and near list `gen`.
FrontScratch ctx_scratch(ov_ctx* ctx, int slot, int gen);
hipError_t launch_fringe(ov_ctx* ctx, int nf, uint8_t* flags, hipStream_t s, int slot = 0, int gen = 0);
hipError_t launch_fringe_in(ov_ctx* ctx, int nf, uint8_t* flags, hipStream_t s, const FrontScratch& fs);
// A new stamp on slot 0 and its near list built from the flags themselves
// (tiles holding a hole), for a fringe pass whose flags came from any hole cut.
hipError_t launch_near_from_flags(ov_ctx* ctx, const uint8_t* flags, hipStream_t s);
// The near list of fs from the flags, under fs's current stamp.
hipError_t launch_near_list_in(ov_ctx* ctx, const uint8_t* flags, hipStream_t s, const FrontScratch& fs);
int build_static_chunks(ov_ctx* ctx, hipStream_t s);
// fused: the write kernel forms the superchunk offsets itself (no scan
// kernel); only for callers whose next hole cut on this slot precedes the
// next compaction (the step executors).
hipError_t launch_compact(ov_ctx* ctx, const uint8_t* flags, int32_t* q_grid, int32_t* q_node,
                          long long capacity, long long* d_count, hipStream_t s, int slot = 0, bool fused = false);
hipError_t launch_compact_in(ov_ctx* ctx, const uint8_t* flags, int32_t* q_grid, int32_t* q_node,
                             long long capacity, long long* d_count, hipStream_t s, const FrontScratch& fs,
                             bool fused);
hipError_t launch_transform(ov_ctx* ctx, const double* poses, const int32_t* q_grid, const int32_t* q_node,
                            const long long* d_count, long long capacity, void* qx, hipStream_t s);
hipError_t launch_donor_search(ov_ctx* ctx, const double* poses, const uint8_t* flags, const int32_t* q_grid,
                               const int32_t* q_node, const void* qx, const long long* d_count,
                               long long capacity, int32_t* donor_grid, int32_t* donor_cell, void* s,
                               int32_t* status, hipStream_t st, int slot = 0);
hipError_t launch_interp(ov_ctx* ctx, const int32_t* donor_grid, const int32_t* donor_cell, const void* s,
                         const long long* d_count, long long capacity, const void* fields, void* out,
                         hipStream_t st);
// The back half of a step (transform, donor search, interpolation when
// fields is non-null) for the step executors: one kernel when back_fused is
// set, else the three launchers above. count_out (nullable) receives the
// step's query count; slot is the step's front-half scratch slot (its stamp
// dates the warm-start entries).
// back_fused = 2 with a deferral queue (defer_items: capacity entries,
// defer_count: four counters, zero before the first step; caller-owned, for
// the back halves of one stream) runs it as two kernels: the walk, and the
// FP64 corrections and brute-force scans of the queries the walk left;
// back_queue takes the one or first kernel's chunks from a work queue whose
// heads are defer_count[2, 4); back_xcd puts runs of that many consecutive
// chunks of the first (or, without the queue, every) round on one XCD.
hipError_t launch_back(ov_ctx* ctx, const double* poses, const uint8_t* flags, const int32_t* q_grid,
                       const int32_t* q_node, void* qx, const long long* d_count, long long capacity,
                       int32_t* donor_grid, int32_t* donor_cell, void* s, int32_t* status, const void* fields,
                       void* out, long long* count_out, hipStream_t st, int slot = 0, int32_t* defer_items = nullptr,
                       unsigned int* defer_count = nullptr);
hipError_t launch_copy_count(long long* dst, const int64_t* src, hipStream_t st);
hipError_t launch_frame_velocity(ov_ctx* ctx, const double* poses, const int32_t* q_grid,
                                 const int32_t* donor_grid, const long long* d_count, long long capacity, void* out,
                                 hipStream_t st);
// setup (control cells, shadows)
int build_control_cells(ov_ctx* ctx, GridHost& g, hipStream_t s);
int build_subbins(ov_ctx* ctx, GridHost& g, const std::vector<unsigned long long>& cnt, hipStream_t s);
int build_shadows(ov_ctx* ctx, GridHost& g, hipStream_t s);
int build_gather_layout(ov_ctx* ctx, GridHost& g, hipStream_t s);

// ---------------------------------------------------------------- device helpers
// Pointers read from the grid table or from LDS carry no address space, so
// loads through them would be flat instructions (which also wait on LDS
// traffic); the library's arrays are all in device memory, and gp() says so.
template <typename T>
using gmem = const __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T>* gp(const T* p) {
  return (gmem<T>*)p;
}

typedef double ov_dv2 __attribute__((ext_vector_type(2)));
// Bin of a coordinate along one axis of a surface triangulation's (y, z)
// grid: the same formula on the host (binning triangle boxes) and on the
// device (binning a node), so that a triangle whose box holds the node is
// listed in the node's bin (the map is monotone in v).
__host__ __device__ __forceinline__ int mesh_bin(double v, double lo, double inv, int n) {
#pragma clang fp contract(off)
  const double t = floor((v - lo) * inv);
  return t < 0.0 ? 0 : (t >= (double)n ? n - 1 : (int)t);
}

// Ray-parity inside test of a closed surface triangulation (the body's
// surface triangles, Sec. 2.2.2): the ray from (x, y, z) along +x crosses
// the surface an odd number of times. Only the triangles of the node's
// (y, z) bin can be crossed. A triangle counts when the node's (y, z) lies
// in its counter-clockwise projection (edge functions > 0, or = 0 on an
// included edge) and the crossing lies beyond x. The edge function of a
// projected edge is evaluated from its endpoint of smaller (y, z) and
// negated for the other direction, so the two triangles of a shared edge
// get exactly opposite values, and an edge is included when it runs toward
// larger z (or, level, toward larger y): a crossing through a shared edge
// or vertex counts once. No contraction into fused multiply-adds: the
// decision is the same, bit for bit, as the reference evaluation order.
__host__ __device__ __forceinline__ double mesh_edge_raw(const double* u, const double* v, double py, double pz) {
#pragma clang fp contract(off)
  const double t0 = (v[1] - u[1]) * (pz - u[2]);
  const double t1 = (v[2] - u[2]) * (py - u[1]);
  return t0 - t1;
}

__host__ __device__ __forceinline__ double mesh_edge(const double* u, const double* v, double py, double pz) {
  if (u[1] < v[1] || (u[1] == v[1] && u[2] < v[2])) return mesh_edge_raw(u, v, py, pz);
  return -mesh_edge_raw(v, u, py, pz);
}

__host__ __device__ __forceinline__ bool mesh_edge_included(const double* u, const double* v) {
#pragma clang fp contract(off)
  const double dz = v[2] - u[2], dy = v[1] - u[1];
  return dz > 0.0 || (dz == 0.0 && dy > 0.0);
}

// Whether the ray from (x, y, z) along +x crosses triangle t (9 doubles:
// a, b, c, already counter-clockwise in the (y, z) projection).
__host__ __device__ __forceinline__ bool mesh_crossed(const double* t, double x, double y, double z) {
#pragma clang fp contract(off)
  const double* a = t;
  const double* b = t + 3;
  const double* c = t + 6;
  const double w0 = mesh_edge(b, c, y, z), w1 = mesh_edge(c, a, y, z), w2 = mesh_edge(a, b, y, z);
  if (!(w0 > 0.0 || (w0 == 0.0 && mesh_edge_included(b, c)))) return false;
  if (!(w1 > 0.0 || (w1 == 0.0 && mesh_edge_included(c, a)))) return false;
  if (!(w2 > 0.0 || (w2 == 0.0 && mesh_edge_included(a, b)))) return false;
  const double den = (w0 + w1) + w2;
  const double num = (w0 * a[0] + w1 * b[0]) + w2 * c[0];
  return num > x * den;
}

// tri: the triangles of each (y, z) bin stored contiguously (9 doubles
// each), already in counter-clockwise projected order, edge-on ones left
// out (both fixed at set-up with the same edge function). Two triangles are
// loaded per round, so that their loads are in flight together (four held
// more registers than they saved).
__host__ __device__ inline bool mesh_parity(const double* tri, const int* start, const double* bx, const double* inv,
                                            const int* n, double x, double y, double z) {
#pragma clang fp contract(off)
  if (x < bx[0] || x > bx[3] || y < bx[1] || y > bx[4] || z < bx[2] || z > bx[5]) return false;
  const int bin = mesh_bin(z, bx[2], inv[1], n[1]) * n[0] + mesh_bin(y, bx[1], inv[0], n[0]);
  const int e1 = start[bin + 1];
  bool odd = false;
  int e = start[bin];
  for (; e + 1 < e1; e += 2) {
    double t[2][9];
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 9; ++k) t[j][k] = tri[9LL * (e + j) + k];
    for (int j = 0; j < 2; ++j) odd ^= mesh_crossed(t[j], x, y, z);
  }
  if (e < e1) odd ^= mesh_crossed(tri + 9LL * e, x, y, z);
  return odd;
}

// The warm-start record of a node with no history.
constexpr unsigned long long kWarmEmpty = 0x000000FFFFFFFFFFULL;  // cell -1, grid 255, stamp 0
constexpr int kStatSlots = 64;
constexpr int kStatStride = 16;  // 128 bytes: one slot per cache line
// This workgroup's slot of the statistics counters.
__device__ __forceinline__ unsigned long long* stat_slot(unsigned long long* stats) {
  return stats + (blockIdx.x & (kStatSlots - 1)) * kStatStride;
}

// The dispatcher hands a launch's workgroups to the chip's XCDs in turn
// (workgroup b to XCD b mod kXcds), and each XCD has its own L2. xcd_rank
// renumbers them so that runs of k consecutive ranks fall on one XCD and the
// runs go to the XCDs in turn: work items taken in rank order then meet their
// k - 1 neighbours in one L2, and every XCD still gets an even mix of the
// whole range. A bijection of [0, nb) when kXcds * k divides nb; otherwise
// (and for k = 0) the launch order is kept.
constexpr int kXcds = 8;
__device__ __forceinline__ long long xcd_rank(long long b, long long nb, int k) {
  if (k <= 0 || nb % ((long long)kXcds * k) != 0) return b;
  const long long x = b % kXcds, l = b / kXcds;
  return ((l / k) * kXcds + x) * k + l % k;
}

typedef float ov_fv4 __attribute__((ext_vector_type(4)));
typedef int ov_iv4 __attribute__((ext_vector_type(4)));

// (x, y, z) of node n from a grid's gather layout: two 16-byte loads.
__device__ __forceinline__ void load_xyz(const GridDev& G, long long n, double& x, double& y, double& z) {
  gmem<ov_dv2>* p = (gmem<ov_dv2>*)gp(G.P) + 2 * n;
  const ov_dv2 a = p[0], b = p[1];
  x = a.x;
  y = a.y;
  z = b.x;
}

__device__ __forceinline__ int grid_of_node(const long long* off, int ngrids, long long n) {
  int lo = 0, hi = ngrids - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= n) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// (ci, cj, ck) of a linear cell index without an integer division: a grid
// has fewer than 2^31 cells, so the FP64 product with the rounded reciprocal
// is within 2^-21 of the exact quotient, and its floor is the quotient or
// one off it (only next to an exact multiple), which one comparison fixes.
__device__ __forceinline__ int div_by(int c, int d, double inv) {
  int q = (int)((double)c * inv);
  if ((long long)q * d > c) --q;
  else if ((long long)(q + 1) * d <= c) ++q;
  return q;
}

__device__ __forceinline__ void cell_ijk(const GridDev& g, long long cell, int& ci, int& cj, int& ck) {
  const int c = (int)cell;
  const int plane = g.nci * g.ncj;
  ck = div_by(c, plane, g.inv_plane);
  const int r = c - ck * plane;
  cj = div_by(r, g.nci, g.inv_nci);
  ci = r - cj * g.nci;
}

// Node of corner c (c0 + 2 c1 + 4 c2) of cell (ci, cj, ck); periodic wrap.
// 32-bit arithmetic: a grid has fewer than 2^31 nodes.
__device__ __forceinline__ long long corner_node(const GridDev& g, int ci, int cj, int ck, int c) {
  int i = ci + (c & 1), j = cj + ((c >> 1) & 1), k = ck + ((c >> 2) & 1);
  i = (i == g.ni) ? 0 : i;
  j = (j == g.nj) ? 0 : j;
  k = (k == g.nk) ? 0 : k;
  return (long long)((unsigned)i + (unsigned)g.ni * ((unsigned)j + (unsigned)g.nj * (unsigned)k));
}

// Padded corner box of a cell (FP64), the same test the fallback scan applies.
__device__ __forceinline__ void cell_box(const GridDev& g, long long cell, double lo[3], double hi[3]) {
  int ci, cj, ck;
  cell_ijk(g, cell, ci, cj, ck);
  for (int d = 0; d < 3; ++d) {
    lo[d] = INFINITY;
    hi[d] = -INFINITY;
  }
  for (int c = 0; c < 8; ++c) {
    long long m = corner_node(g, ci, cj, ck, c);
    double v[3] = {g.X[m], g.Y[m], g.Z[m]};
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], v[d]);
      hi[d] = fmax(hi[d], v[d]);
    }
  }
  double ext = fmax(hi[0] - lo[0], fmax(hi[1] - lo[1], hi[2] - lo[2]));
  double pad = 1e-9 * ext + 1e-300;
  for (int d = 0; d < 3; ++d) {
    lo[d] -= pad;
    hi[d] += pad;
  }
}

// Offset of node m of grid G from the grid's frame centre in inertial axes,
// o = R X (pose p: R row-major, then the centre): FP64 from the FP64
// coordinates, or FP32 from their FP32 roundings (the values of the FP32
// shadows) and the rounded pose. The coordinates come from the packed
// gather layout: one 32-byte record instead of three arrays.
template <typename T>
__device__ __forceinline__ void transform_xyz(const double* p, double X, double Y, double Z, T o[3]) {
  if (sizeof(T) == 8) {
    o[0] = (T)(p[0] * X + p[1] * Y + p[2] * Z);
    o[1] = (T)(p[3] * X + p[4] * Y + p[5] * Z);
    o[2] = (T)(p[6] * X + p[7] * Y + p[8] * Z);
  } else {
    const float Xf = (float)X, Yf = (float)Y, Zf = (float)Z;
    o[0] = (T)((float)p[0] * Xf + (float)p[1] * Yf + (float)p[2] * Zf);
    o[1] = (T)((float)p[3] * Xf + (float)p[4] * Yf + (float)p[5] * Zf);
    o[2] = (T)((float)p[6] * Xf + (float)p[7] * Yf + (float)p[8] * Zf);
  }
}

template <typename T>
__device__ __forceinline__ void transform_node(const GridDev& G, const double* p, long long m, T o[3]) {
  double X, Y, Z;
  load_xyz(G, m, X, Y, Z);
  transform_xyz<T>(p, X, Y, Z, o);
}

// Trilinear interpolation of the 4 fields in cell `cell` of grid B at
// natural coordinates s: weights w_c = prod_d (c_d ? s_d : 1 - s_d) over the
// 8 corners (periodic wrap). Fields: four blocks (field f of node n at
// fields[f * total + n]) or, interleaved, fields[4 n + f] (one 16- or
// 32-byte load per corner).
template <typename T>
__device__ __forceinline__ void interp_point(const GridDev& G, int cell, T s0, T s1, T s2,
                                             const T* __restrict__ fields, long long total, bool interleaved,
                                             T v[4]) {
  int ci, cj, ck;
  cell_ijk(G, cell, ci, cj, ck);
  T w[8];
  long long nd[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    T a = (c & 1) ? s0 : (T)1 - s0;
    T b = (c & 2) ? s1 : (T)1 - s1;
    T d = (c & 4) ? s2 : (T)1 - s2;
    w[c] = a * b * d;
    nd[c] = G.node_off + corner_node(G, ci, cj, ck, c);
  }
  if (interleaved) {
    T acc[4] = {0, 0, 0, 0};
    T q[8][4];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (sizeof(T) == 4) {
        const ov_fv4 x = ((gmem<ov_fv4>*)gp(fields))[nd[c]];
        q[c][0] = (T)x.x;
        q[c][1] = (T)x.y;
        q[c][2] = (T)x.z;
        q[c][3] = (T)x.w;
      } else {
        gmem<ov_dv2>* p = (gmem<ov_dv2>*)gp(fields) + 2 * nd[c];
        const ov_dv2 a = p[0], b = p[1];
        q[c][0] = (T)a.x;
        q[c][1] = (T)a.y;
        q[c][2] = (T)b.x;
        q[c][3] = (T)b.y;
      }
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[f] += w[c] * q[c][f];
      v[f] = acc[f];
    }
    return;
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    gmem<T>* F = gp(fields) + (long long)f * total;
    T acc = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc += w[c] * F[nd[c]];
    v[f] = acc;
  }
}

// A velocity's components turned from donor frame B into receiver frame A:
// v <- R_A^T (R_B v), with R the rotation of each pose (row-major, the pose's
// first 9 values); formed in FP64.
template <typename T>
__device__ __forceinline__ void frame_rotate(const double* pa, const double* pb, T v[3]) {
  const double u0 = (double)v[0], u1 = (double)v[1], u2 = (double)v[2];
  double w[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] = pb[3 * i] * u0 + pb[3 * i + 1] * u1 + pb[3 * i + 2] * u2;
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] = (T)(pa[i] * w[0] + pa[3 + i] * w[1] + pa[6 + i] * w[2]);
}

__device__ __forceinline__ int bin_axis(const GridDev& g, int d, double v) {
  double t = floor((v - g.blo[d]) * g.binv[d]);
  if (!(t >= 0.0)) return 0;  // also NaN
  if (t >= (double)g.nb[d]) return g.nb[d] - 1;
  return (int)t;
}

// Sub-bins of a split control cell: kSubBins per axis.
constexpr int kSubBins = 4;
constexpr long long kSplitList = 128;

// Sub-bin coordinate along axis d of v inside bin `bin` of that axis. The
// same product as bin_axis, scaled by kSubBins (exact), so a point inside a
// cell's box falls in a sub-bin the cell was listed in.
__device__ __forceinline__ int sub_axis(const GridDev& g, int d, double v, int bin) {
  const double t = floor((v - g.blo[d]) * g.binv[d] * (double)kSubBins) - (double)kSubBins * bin;
  if (!(t >= 0.0)) return 0;  // also NaN
  return t >= (double)(kSubBins - 1) ? kSubBins - 1 : (int)t;
}

// The candidate donor cells of the control cell (or sub-bin) holding xi:
// entries [e0, e1) of the returned array, ascending.
__device__ __forceinline__ const int* control_list(const GridDev& G, const double xi[3], long long& e0,
                                                   long long& e1) {
  const int bx = bin_axis(G, 0, xi[0]), by = bin_axis(G, 1, xi[1]), bz = bin_axis(G, 2, xi[2]);
  const long long b = bx + (long long)G.nb[0] * (by + (long long)G.nb[1] * bz);
  const int sb = G.bsub ? gp(G.bsub)[b] : -1;
  if (sb < 0) {
    e0 = gp(G.bstart)[b];
    e1 = gp(G.bstart)[b + 1];
    return G.bcells;
  }
  const long long k = sb + sub_axis(G, 0, xi[0], bx) +
                      kSubBins * (sub_axis(G, 1, xi[1], by) + kSubBins * sub_axis(G, 2, xi[2], bz));
  e0 = gp(G.sstart)[k];
  e1 = gp(G.sstart)[k + 1];
  return G.scells;
}

}  // namespace ov
