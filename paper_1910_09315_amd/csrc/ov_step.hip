// Step kernels of the overset grid assembly on gfx950: hole cutting,
// query-point marking, ordered compaction, query transform, trilinear
// interpolation; plus the C-ABI entry points of the step (argument checks,
// then one or more launches on the caller's stream; nothing allocates or
// synchronises).
//
// Paper: Hedayat & Borazjani, arXiv:1910.09315. Hole cutting Sec. 2.2.2 and
// Sec. 2.4 item 2; query points Sec. 2.2.3 item 1 and Alg. 1; coordinate
// packets Sec. 2.2.3 item 6; interpolation Sec. 2.2.6.
#include <hip/hip_runtime.h>

#include <climits>

#include "ov_internal.h"

namespace ov {

// ================================================================ hole cut
// Per-launch copy of what every node needs: grid poses, node offsets and
// coordinate pointers, and the list of grids that carry a blank region.
struct HoleLds {
  double pose[kMaxGrids][12];
  float posef[kMaxGrids][12];
  float prmf[kMaxGrids][6];  // FP32 shape constants: see holecut_stage
  double prm[kMaxGrids][3];
  double cull[kMaxGrids];
  float cullf[kMaxGrids];  // FP32 cull radius^2, widened for FP32 rounding
  long long off[kMaxGrids + 1];
  const void* X[kMaxGrids];
  const void* Y[kMaxGrids];
  const void* Z[kMaxGrids];
  int kind[kMaxGrids];
  int outer[kMaxGrids];
  unsigned long long allmask;  // every grid with a blank region
  double box[kMaxGrids][6];    // blank region's body-frame box (lo xyz, hi xyz)
  double rad[kMaxGrids];       // radius of the sphere about the origin enclosing it
};

// Body-frame box of grid G's blank region (lo xyz, hi xyz; zeros if none).
__device__ __forceinline__ void region_box(const GridDev& G, double* box) {
  const double* q = G.blank_prm;
  double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
  if (G.blank_kind == OV_BLANK_CYL) {
    lo[0] = lo[1] = -q[0];
    hi[0] = hi[1] = q[0];
    lo[2] = q[1];
    hi[2] = q[2];
  } else if (G.blank_kind == OV_BLANK_SPHERE) {
    lo[0] = lo[1] = lo[2] = -q[0];
    hi[0] = hi[1] = hi[2] = q[0];
  } else if (G.blank_kind == OV_BLANK_ELLIPSOID) {
    for (int d = 0; d < 3; ++d) {
      lo[d] = -q[d];
      hi[d] = q[d];
    }
  } else if (G.blank_kind == OV_BLANK_MESH) {
    for (int d = 0; d < 3; ++d) {
      lo[d] = G.mbox[d];
      hi[d] = G.mbox[3 + d];
    }
  }
  for (int d = 0; d < 3; ++d) {
    box[d] = lo[d];
    box[3 + d] = hi[d];
  }
}

template <typename CT>
__device__ __forceinline__ void holecut_stage(HoleLds& L, const GridDev* __restrict__ grids, int ngrids,
                                              const double* __restrict__ poses) {
  for (int i = threadIdx.x; i < ngrids * 12; i += blockDim.x) {
    L.pose[i / 12][i % 12] = poses[i];
    L.posef[i / 12][i % 12] = (float)poses[i];
  }
  for (int g = threadIdx.x; g < ngrids; g += blockDim.x) {
    const GridDev& G = grids[g];
    L.off[g] = G.node_off;
    L.kind[g] = G.blank_kind;
    L.outer[g] = G.has_outer;
    L.cull[g] = G.cull_r2;
    L.cullf[g] = (float)G.cull_r2 * 1.0001f + 1e-30f;
    L.prm[g][0] = G.blank_prm[0];
    L.prm[g][1] = G.blank_prm[1];
    L.prm[g][2] = G.blank_prm[2];
    // sphere / cylinder: 1/r^2, -, -, 1/r, z0, z1 ; ellipsoid: 1/a, 1/b, 1/c
    const double* q = G.blank_prm;
    if (G.blank_kind == OV_BLANK_ELLIPSOID) {
      L.prmf[g][0] = (float)(1.0 / q[0]);
      L.prmf[g][1] = (float)(1.0 / q[1]);
      L.prmf[g][2] = (float)(1.0 / q[2]);
    } else if (G.blank_kind == OV_BLANK_MESH) {
      // the surface's box padded far beyond FP32 rounding of a body-frame
      // position: outside it a node is decided in FP32, inside it in FP64
      const double* b = G.mbox;
      const double pad = 1e-3 * fmax(b[3] - b[0], fmax(b[4] - b[1], b[5] - b[2])) + 1e-5;
      for (int d = 0; d < 3; ++d) {
        L.prmf[g][d] = (float)(b[d] - pad);
        L.prmf[g][3 + d] = (float)(b[3 + d] + pad);
      }
    } else if (G.blank_kind == OV_BLANK_SPHERE || G.blank_kind == OV_BLANK_CYL) {
      L.prmf[g][0] = (float)(1.0 / (q[0] * q[0]));
      L.prmf[g][3] = (float)(1.0 / q[0]);
      L.prmf[g][4] = (float)q[1];
      L.prmf[g][5] = (float)q[2];
    }
    if (sizeof(CT) == 4) {
      L.X[g] = G.Xf;
      L.Y[g] = G.Yf;
      L.Z[g] = G.Zf;
    } else {
      L.X[g] = G.X;
      L.Y[g] = G.Y;
      L.Z[g] = G.Z;
    }
    if (g == ngrids - 1) L.off[ngrids] = G.node_off + G.nnodes;
    L.rad[g] = sqrt(G.cull_r2);
    region_box(G, L.box[g]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int g = 0; g < ngrids; ++g)
      if (L.kind[g] != OV_BLANK_NONE) m |= 1ull << g;
    L.allmask = m;
  }
  __syncthreads();
}

// What the sub-tile cull needs of every grid, staged in LDS: pose, the blank
// region's body-frame box and enclosing radius, and the grids that have one.
struct MaskLds {
  double pose[kMaxGrids][12];
  double box[kMaxGrids][6];
  double rad[kMaxGrids];
  unsigned long long allmask;
};

__device__ __forceinline__ void mask_stage(MaskLds& L, const GridDev* __restrict__ grids, int ngrids,
                                           const double* __restrict__ poses) {
  for (int i = threadIdx.x; i < ngrids * 12; i += blockDim.x) L.pose[i / 12][i % 12] = poses[i];
  if (threadIdx.x < 64) {
    const int g = threadIdx.x;
    bool has = false;
    if (g < ngrids) {
      const GridDev& G = grids[g];
      L.rad[g] = sqrt(G.cull_r2);
      region_box(G, L.box[g]);
      has = G.blank_kind != OV_BLANK_NONE;
    }
    const unsigned long long m = __ballot(has);
    if (g == 0) L.allmask = m;
  }
  __syncthreads();
}

// Signed, scale-free inside measure of a body-frame point in FP32: < 0
// strictly inside. For the cylinder the radial and axial conditions are
// combined as a max. c: the FP32 shape constants of holecut_stage.
__device__ __forceinline__ float blank_measure_f32(int kind, const float* c, float x, float y, float z) {
  if (kind == OV_BLANK_SPHERE) return (x * x + y * y + z * z) * c[0] - 1.f;
  if (kind == OV_BLANK_ELLIPSOID) {
    float u = x * c[0], v = y * c[1], w = z * c[2];
    return u * u + v * v + w * w - 1.f;
  }
  float fr = (x * x + y * y) * c[0] - 1.f;
  float fz = fmaxf((c[4] - z) * c[3], (z - c[5]) * c[3]);
  return fmaxf(fr, fz);
}

__device__ __forceinline__ bool blank_inside_fp64(int kind, const double* prm, double x, double y, double z) {
#pragma clang fp contract(off)
  if (kind == OV_BLANK_CYL) {
    double r = prm[0];
    return (x * x + y * y) < r * r && z >= prm[1] && z <= prm[2];
  }
  if (kind == OV_BLANK_SPHERE) return (x * x + y * y + z * z) < prm[0] * prm[0];
  double u = x / prm[0], v = y / prm[1], w = z / prm[2];
  return (u * u + v * v + w * w) < 1.0;
}

// The ray-parity test of a triangulated blank surface: a node in a voxel
// that no triangle's (padded) box meets takes the voxel's precomputed
// status (the surface does not pass between it and the voxel's centre, where
// the same test was evaluated at set-up); a node in a voxel the surface may
// pass through runs the test on the triangles of its (y, z) bin.
// Voxel status of a body-frame point (clamped into the voxel grid).
__device__ __forceinline__ int mesh_voxel(const GridDev& G, double x, double y, double z) {
  const double* bx = G.mbox;
  return G.mvox[(mesh_bin(z, bx[2], G.mvinv[2], G.mvn[2]) * G.mvn[1] + mesh_bin(y, bx[1], G.mvinv[1], G.mvn[1])) *
                    G.mvn[0] +
                mesh_bin(x, bx[0], G.mvinv[0], G.mvn[0])];
}

__device__ __noinline__ bool mesh_inside(const GridDev& G, double x, double y, double z) {
  const double* bx = G.mbox;
  if (x < bx[0] || x > bx[3] || y < bx[1] || y > bx[4] || z < bx[2] || z > bx[5]) return false;
  const int v = mesh_voxel(G, x, y, z);
  if (v != 2) return v == 1;
  return mesh_parity(G.mtri, G.mstart, bx, G.minv, G.mn, x, y, z);
}

// FP64 decision for one node of grid A at world position w: first blanking
// grid (ascending grid id, among the bits of mask) or -1. The body-frame
// position is formed without fused multiply-adds, in the reference order.
// CHEAP: a triangulated region whose voxel the surface may cross is not
// tested here; the node's decision is deferred (kDeferNode) to a balanced
// pass of the whole workgroup.
constexpr int kDeferNode = -2;

template <bool MESH, bool CHEAP = false>
__device__ __forceinline__ int holecut_fp64(const HoleLds& L, const GridDev* __restrict__ grids, int A,
                                            const double w[3], unsigned long long mask) {
#pragma clang fp contract(off)
  mask &= ~(1ull << A);
  while (mask) {
    const int B = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    const double* p = L.pose[B];
    double d0 = w[0] - p[9], d1 = w[1] - p[10], d2 = w[2] - p[11];
    if (d0 * d0 + d1 * d1 + d2 * d2 >= L.cull[B]) continue;
    double x = (p[0] * d0 + p[3] * d1) + p[6] * d2;
    double y = (p[1] * d0 + p[4] * d1) + p[7] * d2;
    double z = (p[2] * d0 + p[5] * d1) + p[8] * d2;
    bool in;
    if constexpr (MESH) {
      if (L.kind[B] != OV_BLANK_MESH) {
        in = blank_inside_fp64(L.kind[B], L.prm[B], x, y, z);
      } else if (CHEAP) {
        const double* bx = L.box[B];
        const bool in_box = !(x < bx[0] || x > bx[3] || y < bx[1] || y > bx[4] || z < bx[2] || z > bx[5]);
        const int v = in_box ? mesh_voxel(grids[B], x, y, z) : 0;
        if (v == 2) return kDeferNode;
        in = v == 1;
      } else {
        in = mesh_inside(grids[B], x, y, z);
      }
    } else {
      in = blank_inside_fp64(L.kind[B], L.prm[B], x, y, z);
    }
    if (in) return B;
  }
  return -1;
}

// World position of a node, ((R_i0 X + R_i1 Y) + R_i2 Z) + c_i, without
// fused multiply-adds (the reference order).
__device__ __forceinline__ void world_exact(const double* pa, double X, double Y, double Z, double w[3]) {
#pragma clang fp contract(off)
  for (int i = 0; i < 3; ++i) w[i] = ((pa[3 * i] * X + pa[3 * i + 1] * Y) + pa[3 * i + 2] * Z) + pa[9 + i];
}

// FP32 guard band: nodes whose FP32 inside measure is within this of the
// surface are decided again in FP64 from the FP64 coordinates.
constexpr float kHoleGuard = 1e-3f;

// Hole decision of one node of grid A: the blank regions of the grids in
// mask (a superset of those that can contain it) are tested in ascending
// grid id; the first that contains the node is its cause. In FP32, a node
// within the guard band of a surface is decided again in FP64.
// MESH: some grid's blank region is a triangulation (a variant of its own,
// so that the other kernels keep their registers).
// DEFER: return kDeferNode instead of running a triangulation's parity
// test (the caller decides those nodes in a balanced pass).
template <typename CT, bool MESH, bool DEFER = false>
__device__ __forceinline__ int holecut_node(const HoleLds& L, const GridDev* __restrict__ grids, int A, long long m,
                                            CT X, CT Y, CT Z, unsigned long long mask) {
  const double* pa = L.pose[A];
  if (sizeof(CT) == 8) {
    double w[3];
    world_exact(pa, (double)X, (double)Y, (double)Z, w);
    return holecut_fp64<MESH, DEFER>(L, grids, A, w, mask);
  }
  const float* pf = L.posef[A];
  const float Xf = (float)X, Yf = (float)Y, Zf = (float)Z;
  float w0 = pf[0] * Xf + pf[1] * Yf + pf[2] * Zf + pf[9];
  float w1 = pf[3] * Xf + pf[4] * Yf + pf[5] * Zf + pf[10];
  float w2 = pf[6] * Xf + pf[7] * Yf + pf[8] * Zf + pf[11];
  bool unsure = false;
  int cause = -1;
  for (unsigned long long mm = mask & ~(1ull << A); mm; mm &= mm - 1) {
    const int B = __ffsll((long long)mm) - 1;
    const float* p = L.posef[B];
    float d0 = w0 - p[9], d1 = w1 - p[10], d2 = w2 - p[11];
    if (d0 * d0 + d1 * d1 + d2 * d2 >= L.cullf[B]) continue;
    float x = p[0] * d0 + p[3] * d1 + p[6] * d2;
    float y = p[1] * d0 + p[4] * d1 + p[7] * d2;
    float z = p[2] * d0 + p[5] * d1 + p[8] * d2;
    // a triangulated surface: outside its padded box, or in a voxel the
    // surface does not reach, decided in FP32 (the voxel's status holds within
    // a padding far above FP32 error); otherwise in FP64
    const float* c = L.prmf[B];
    float f;
    if (!MESH || L.kind[B] != OV_BLANK_MESH) {
      f = blank_measure_f32(L.kind[B], c, x, y, z);
    } else if (x < c[0] || x > c[3] || y < c[1] || y > c[4] || z < c[2] || z > c[5]) {
      f = 1.f;
    } else {
      // (only strictly inside the surface's box: near its faces the FP64
      // test decides)
      const double* bx = L.box[B];
      const double xd = x, yd = y, zd = z;
      const bool in_box = xd > bx[0] && xd < bx[3] && yd > bx[1] && yd < bx[4] && zd > bx[2] && zd < bx[5];
      const int v = in_box ? mesh_voxel(grids[B], xd, yd, zd) : 2;
      f = v == 0 ? 1.f : v == 1 ? -1.f : 0.f;
    }
    if (fabsf(f) < kHoleGuard) {
      unsure = true;
      break;
    }
    if (f < 0.f) {
      cause = B;
      break;
    }
  }
  if (unsure) {
    const GridDev& G = grids[A];
    double Xd = gp(G.X)[m], Yd = gp(G.Y)[m], Zd = gp(G.Z)[m];
    double w[3];
    world_exact(pa, Xd, Yd, Zd, w);
    cause = holecut_fp64<MESH, DEFER>(L, grids, A, w, mask);
  }
  return cause;
}

// The full FP64 decision of node m of grid A from its FP64 coordinates.
template <bool MESH>
__device__ __forceinline__ int holecut_node_exact(const HoleLds& L, const GridDev* __restrict__ grids, int A,
                                                  long long m, unsigned long long mask) {
  const GridDev& G = grids[A];
  double w[3];
  world_exact(L.pose[A], gp(G.X)[m], gp(G.Y)[m], gp(G.Z)[m], w);
  return holecut_fp64<MESH>(L, grids, A, w, mask);
}

// Flag byte of a node given its hole cause (-1: none). Holes mark their
// fringe tile in the tile map; nodes of grids with outer layers compute their
// (i, j, k) to mark the outer-boundary query layers (a fixed set per grid).
// Grid geometry kept in registers by loops that store flag bytes (a byte
// store may alias anything, so fields read through a GridDev reference would
// be re-loaded after every store).
struct GeomR {
  int ni, nj, nk, per, tiles_i, tiles_j;
  int o0, o1, o2, o3, o4, o5;
  long long tile_off;
  __device__ __forceinline__ explicit GeomR(const GridDev& G)
      : ni(G.ni), nj(G.nj), nk(G.nk), per(G.per), tiles_i(G.tiles_i), tiles_j(G.tiles_j), o0(G.outer[0]),
        o1(G.outer[1]), o2(G.outer[2]), o3(G.outer[3]), o4(G.outer[4]), o5(G.outer[5]), tile_off(G.tile_off) {}
  __device__ __forceinline__ bool on_outer(int i, int j, int k) const {
    return i < o0 || i >= ni - o1 || j < o2 || j >= nj - o3 || k < o4 || k >= nk - o5;
  }
};

__device__ __forceinline__ uint8_t node_flag(const GeomR& G, long long m, int cause, unsigned int* tile_hole,
                                             unsigned int stamp) {
  long long plane = (long long)G.ni * G.nj;
  int k = (int)(m / plane);
  long long r = m - (long long)k * plane;
  int j = (int)(r / G.ni);
  int i = (int)(r - (long long)j * G.ni);
  if (cause >= 0) {
    tile_hole[G.tile_off + (i >> 6) + (long long)G.tiles_i * ((j >> 3) + (long long)G.tiles_j * (k >> 3))] = stamp;
    return (uint8_t)(kHole | (cause << 2));
  }
  return G.on_outer(i, j, k) ? (uint8_t)(kFringe | (OV_CAUSE_BOUNDARY << 2)) : (uint8_t)OV_STATE_FIELD;
}

// Work is split into chunks of blockDim * W * R consecutive nodes that never
// straddle two grids, so the grid of a chunk is uniform across the block.
// Each lane loads R vectors of W consecutive nodes (16 bytes) per coordinate
// array before testing any node, keeping 3 R 16-byte loads in flight.
template <typename CT>
struct Vec16;
typedef double ov_d2 __attribute__((ext_vector_type(2)));
typedef float ov_f4 __attribute__((ext_vector_type(4)));
template <>
struct Vec16<double> {
  typedef ov_d2 type;
  static constexpr int W = 2;
};
template <>
struct Vec16<float> {
  typedef ov_f4 type;
  static constexpr int W = 4;
};

template <typename CT, int R>
__global__ void __launch_bounds__(1024) k_holecut(const GridDev* __restrict__ grids, int ngrids,
                                                 const double* __restrict__ poses, uint8_t* __restrict__ flags,
                                                 long long total_chunks, unsigned int* __restrict__ tile_hole,
                                                 const unsigned int* __restrict__ d_stamp,
                                                 unsigned long long* __restrict__ stats) {
  typedef typename Vec16<CT>::type V;
  constexpr int W = Vec16<CT>::W;
  __shared__ HoleLds L;
  __shared__ long long coff[kMaxGrids + 1];  // first chunk of each grid
  const unsigned int stamp = *d_stamp;
  holecut_stage<CT>(L, grids, ngrids, poses);
  const long long span = (long long)blockDim.x * W * R;
  if (threadIdx.x == 0) {
    long long c = 0;
    for (int g = 0; g < ngrids; ++g) {
      coff[g] = c;
      c += (L.off[g + 1] - L.off[g] + span - 1) / span;
    }
    coff[ngrids] = c;
    if (blockIdx.x == 0) {
      atomicAdd(&stat_slot(stats)[OV_STAT_HOLECUT_NODES_READ], (unsigned long long)L.off[ngrids]);
      atomicAdd(&stat_slot(stats)[OV_STAT_HOLECUT_CALLS], 1ULL);
    }
  }
  __syncthreads();
  for (long long ch = blockIdx.x; ch < total_chunks; ch += gridDim.x) {
    const int A = grid_of_node(coff, ngrids, ch);
    const long long nn = L.off[A + 1] - L.off[A];
    const long long m0 = (ch - coff[A]) * span + (long long)threadIdx.x * W;
    gmem<CT>* Xa = gp((const CT*)L.X[A]);
    gmem<CT>* Ya = gp((const CT*)L.Y[A]);
    gmem<CT>* Za = gp((const CT*)L.Z[A]);
    uint8_t* fa = flags + L.off[A];
    const GeomR GR(grids[A]);
    const bool outerA = L.outer[A] != 0;
    CT X[R][W], Y[R][W], Z[R][W];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long m = m0 + (long long)r * blockDim.x * W;
      if (m + W <= nn) {
        V x = __builtin_nontemporal_load((gmem<V>*)(Xa + m));
        V y = __builtin_nontemporal_load((gmem<V>*)(Ya + m));
        V z = __builtin_nontemporal_load((gmem<V>*)(Za + m));
#pragma unroll
        for (int w = 0; w < W; ++w) {
          X[r][w] = x[w];
          Y[r][w] = y[w];
          Z[r][w] = z[w];
        }
      } else {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          if (m + w < nn) {
            X[r][w] = Xa[m + w];
            Y[r][w] = Ya[m + w];
            Z[r][w] = Za[m + w];
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long m = m0 + (long long)r * blockDim.x * W;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (m + w >= nn) continue;
        int cause = holecut_node<CT, true>(L, grids, A, m + w, X[r][w], Y[r][w], Z[r][w], L.allmask);
        fa[m + w] = (cause < 0 && !outerA) ? (uint8_t)OV_STATE_FIELD : node_flag(GR, m + w, cause, tile_hole, stamp);
      }
    }
  }
}

static_assert(kTileI == 64 && kTileJ == 8 && kTileK == 8 && 256 * 16 == kTileI * kTileJ * kTileK,
              "a 256-thread block covers a tile with 16 bytes per thread");

// Starts a step of the front half: a new stamp, empty near and chunk lists.
// Later kernels of the hole cut read the stamp (stream order).
// `counter` numbers the steps of the context on the device (stamp = 0: the
// step takes the next number); a nonzero stamp was numbered by the host in
// issue order (the by-step executor, whose hole cuts may run in any order)
// and only raises the counter. `d_stamp` is the stamp of the scratch slot
// this step uses (separate slots let the stages of one step overlap those of
// others).
// `high` (0 or kStampHigh) keeps the stamps of two counters apart: the hole
// cut's starts count on one, the fringe call of the C ABI (which starts its
// own lists from the flags it is given) on another, so that the hole cut's
// counter advances once per step (the warm start dates its records by it).
__device__ __forceinline__ void k_begin_step_body(unsigned int stamp, unsigned int* counter, unsigned int* d_stamp,
                                                  int32_t* near_count, int32_t* chunk_list_count,
                                                  unsigned int high = 0u) {
  unsigned int v = stamp;
  if (v == 0u) {
    v = stamp_after(*counter);
    *counter = v;
  } else {
    atomicMax(counter, v);
  }
  *d_stamp = v | high;
  *near_count = 0;
  *chunk_list_count = 0;
}

__global__ void k_begin_step(unsigned int stamp, unsigned int* __restrict__ counter, unsigned int* __restrict__ d_stamp,
                             int32_t* __restrict__ near_count, int32_t* __restrict__ chunk_list_count,
                             int32_t* __restrict__ super_counts, long long n_super_counts, unsigned int high) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    k_begin_step_body(stamp, counter, d_stamp, near_count, chunk_list_count, high);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_super_counts;
       i += (long long)gridDim.x * blockDim.x)
    super_counts[i] = 0;
}

// Tile index along one axis holding the node `which` positions from tile t:
// 0 = kMaxNf before its first node, 1 = one before, 2 = the tile itself,
// 3 = one after its last node, 4 = kMaxNf after (wrapped on a periodic axis,
// clipped otherwise). Buffer nodes lie within kMaxNf nodes of their hole,
// so these tiles hold every buffer node of a hole in tile t, also where the
// last tile of a periodic axis is thinner than kMaxNf.
__device__ __forceinline__ int reach_tile(int t, int which, int n, int size, bool per) {
  const int i0 = t * size, i1 = min(n, i0 + size) - 1;
  int v = which == 0 ? i0 - kMaxNf : which == 1 ? i0 - 1 : which == 2 ? i0 : which == 3 ? i1 + 1 : i1 + kMaxNf;
  if (per) {
    v %= n;
    if (v < 0) v += n;
  } else {
    v = min(max(v, 0), n - 1);
  }
  return v / size;
}

// Puts combination e (< 125) of the reach tiles of tile (ti, tj, tk) of
// grid g on the near list, once per stamp, as its (grid, tile i, j, k).
__device__ __forceinline__ void mark_near(int e, int g, int ti, int tj, int tk, int ni, int nj, int nk, int per, int tiles_i,
                                          int tiles_j, long long tile_off, unsigned int stamp,
                                          unsigned int* __restrict__ tile_near, int4* __restrict__ near_list,
                                          int32_t* __restrict__ near_count) {
  const int x = reach_tile(ti, e % 5, ni, kTileI, per & 1);
  const int y = reach_tile(tj, (e / 5) % 5, nj, kTileJ, per & 2);
  const int z = reach_tile(tk, e / 25, nk, kTileK, per & 4);
  const long long n = tile_off + x + (long long)tiles_i * (y + (long long)tiles_j * z);
  if (atomicExch(&tile_near[n], stamp) != stamp) near_list[atomicAdd(near_count, 1)] = make_int4(g, x, y, z);
}

// The tiles along one axis that hold a position within kMaxNf of the range
// [lo, hi] (which lies inside one tile), as a run of `count` consecutive
// tiles from `first` (modulo the tile count on a periodic axis). Where the
// padded range could come round to its first tile again (an axis hardly
// longer than it), every tile of the axis.
__device__ __forceinline__ void reach_run(int lo, int hi, int n, int size, bool per, int& first, int& count) {
  const int nt = (n + size - 1) / size;
  if (per) {
    if (hi - lo + 1 + 2 * kMaxNf + size > n) {
      first = 0;
      count = nt;
      return;
    }
    const int a = lo - kMaxNf < 0 ? lo - kMaxNf + n : lo - kMaxNf;
    const int b = hi + kMaxNf >= n ? hi + kMaxNf - n : hi + kMaxNf;
    first = a / size;
    count = (b / size - first + nt) % nt + 1;
  } else {
    first = max(lo - kMaxNf, 0) / size;
    count = min(hi + kMaxNf, n - 1) / size - first + 1;
  }
}

// The holes of a sub-tile as a box of node indices (lo/hi per axis; lo >
// hi when there are none), and the near-list entries it gives: every tile
// holding a node within kMaxNf of the box, which holds every buffer node
// the sub-tile's holes can make.
struct HoleBox {
  int lo[3], hi[3];
};

__device__ __forceinline__ void hole_box_wave(HoleBox& b) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      b.lo[d] = min(b.lo[d], __shfl_xor(b.lo[d], o, 64));
      b.hi[d] = max(b.hi[d], __shfl_xor(b.hi[d], o, 64));
    }
}

// Lanes `lane` of `width` put entry e = lane, lane + width, ... of the box's
// runs along i, j and k on the near list (once per stamp). Every lane of a
// wavefront calls it with the same box; the entries a wavefront claims are
// appended with one atomic on the list's count.
__device__ __forceinline__ void mark_near_box(const HoleBox& b, int lane, int width, int g, int ni, int nj, int nk,
                                              int per, int tiles_i, int tiles_j, long long tile_off,
                                              unsigned int stamp, unsigned int* __restrict__ tile_near,
                                              int4* __restrict__ near_list, int32_t* __restrict__ near_count) {
  int fi, ci, fj, cj, fk, ck;
  reach_run(b.lo[0], b.hi[0], ni, kTileI, per & 1, fi, ci);
  reach_run(b.lo[1], b.hi[1], nj, kTileJ, per & 2, fj, cj);
  reach_run(b.lo[2], b.hi[2], nk, kTileK, per & 4, fk, ck);
  const int tiles_k = (nk + kTileK - 1) / kTileK;
  const int total = ci * cj * ck;
  const int wl = (int)(threadIdx.x & 63);
  for (int e0 = 0; e0 < total; e0 += width) {
    const int e = e0 + lane;
    int x = 0, y = 0, z = 0;
    bool fresh = false;
    if (e < total) {
      x = fi + e % ci;
      y = fj + (e / ci) % cj;
      z = fk + e / (ci * cj);
      x = x >= tiles_i ? x - tiles_i : x;
      y = y >= tiles_j ? y - tiles_j : y;
      z = z >= tiles_k ? z - tiles_k : z;
      const long long n = tile_off + x + (long long)tiles_i * (y + (long long)tiles_j * z);
      fresh = atomicExch(&tile_near[n], stamp) != stamp;
    }
    const unsigned long long fm = __ballot(fresh);
    if (fm) {
      const int leader = __ffsll((long long)fm) - 1;
      int base = 0;
      if (wl == leader) base = atomicAdd(near_count, (int)__popcll(fm));
      base = __shfl(base, leader, 64);
      if (fresh) near_list[base + (int)__popcll(fm & ((1ull << wl) - 1ull))] = make_int4(g, x, y, z);
    }
  }
}

// Which blank regions may reach sub-tile `sub` (bit B set: grid B's region
// may contain a node of it). The sub-tile's bounding sphere (radius w),
// placed at its grid's pose, is tested against the sphere about grid B's
// origin that encloses B's region (radius R), then against the region's box
// in B's body frame. Both tests are padded by a relative 1e-9 of the lengths
// involved plus 1e-12, far beyond FP64 rounding, so no node the exact test
// would blank is ever culled. The sphere test compares squared distances:
// with centre distance d, B is kept while d <= K = (R + w)(1 + 3e-9) + 2e-12,
// which exceeds ((R + w)(1 + 1e-9) + 1e-12) / (1 - 1e-9), the bound of the
// test d <= R + w + 1e-9 (w + d + R) + 1e-12; the box test then uses the
// padded radius w + 1e-9 (w + K + R) + 1e-12, at least the one the distance
// itself would give.
template <class LDS>
__device__ __forceinline__ unsigned long long sub_mask(const LDS& L, int A, double4 sp) {
  const double* pa = L.pose[A];
  const double w0 = pa[0] * sp.x + pa[1] * sp.y + pa[2] * sp.z + pa[9];
  const double w1 = pa[3] * sp.x + pa[4] * sp.y + pa[5] * sp.z + pa[10];
  const double w2 = pa[6] * sp.x + pa[7] * sp.y + pa[8] * sp.z + pa[11];
  unsigned long long mask = 0;
  for (unsigned long long mm = L.allmask & ~(1ull << A); mm; mm &= mm - 1) {
    const int B = __ffsll((long long)mm) - 1;
    const double* p = L.pose[B];
    const double d0 = w0 - p[9], d1 = w1 - p[10], d2 = w2 - p[11];
    const double K = (L.rad[B] + sp.w) * (1.0 + 3e-9) + 2e-12;
    if (d0 * d0 + d1 * d1 + d2 * d2 > K * K) continue;
    const double r = sp.w + 1e-9 * (sp.w + K + L.rad[B]) + 1e-12;
    const double x = p[0] * d0 + p[3] * d1 + p[6] * d2;
    const double y = p[1] * d0 + p[4] * d1 + p[7] * d2;
    const double z = p[2] * d0 + p[5] * d1 + p[8] * d2;
    const double ex = fmax(fmax(L.box[B][0] - x, x - L.box[B][3]), 0.0);
    const double ey = fmax(fmax(L.box[B][1] - y, y - L.box[B][4]), 0.0);
    const double ez = fmax(fmax(L.box[B][2] - z, z - L.box[B][5]), 0.0);
    if (ex * ex + ey * ey + ez * ez <= r * r) mask |= 1ull << B;
  }
  return mask;
}

// The start kernel's share of the cull (OV_OPT_HOLECUT_LIST): mask chunk c
// (kMaskChunk consecutive sub-tiles, one per thread of a 256-thread block)
// for c = bid, bid + nblocks, ...: every sub-tile's mask, and the chunk's
// number of candidates (sub-tiles with a non-zero mask).
__device__ __forceinline__ void mask_chunks(const MaskLds& L, const double4* __restrict__ spheres,
                                            const int4* __restrict__ tile_info, long long nsub,
                                            unsigned long long* __restrict__ sub_mask_out,
                                            int32_t* __restrict__ mask_counts, long long nmc, long long bid,
                                            long long nblocks) {
  static_assert(kMaskChunk == 256, "one sub-tile per thread of a 256-thread block");
  __shared__ int wcount[4];
  for (long long c = bid; c < nmc; c += nblocks) {
    const long long sub = c * kMaskChunk + threadIdx.x;
    unsigned long long m = 0;
    if (sub < nsub) {
      m = sub_mask(L, tile_info[sub / kSubPerTile].x, spheres[sub]);
      sub_mask_out[sub] = m;
    }
    const int wc = (int)__popcll(__ballot(m != 0ull));
    if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = wc;
    __syncthreads();
    if (threadIdx.x == 0) mask_counts[c] = wcount[0] + wcount[1] + wcount[2] + wcount[3];
    __syncthreads();  // wcount is rewritten by the next chunk
  }
}

// Geometry of every grid for the tile kernels, staged in LDS.
struct TileGeo {
  int ni, nj, nk, per, tiles_i, tiles_j;
  int o[6];
  long long tile_off;
};

__device__ __forceinline__ void stage_tile_geo(TileGeo* tg, const GridDev* __restrict__ grids, int ngrids) {
  for (int g = threadIdx.x; g < ngrids; g += blockDim.x) {
    const GridDev& G = grids[g];
    TileGeo t;
    t.ni = G.ni;
    t.nj = G.nj;
    t.nk = G.nk;
    t.per = G.per;
    t.tiles_i = G.tiles_i;
    t.tiles_j = G.tiles_j;
    for (int f = 0; f < 6; ++f) t.o[f] = G.outer[f];
    t.tile_off = G.tile_off;
    tg[g] = t;
  }
}

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
  unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// The cull of the step's sub-tiles, done by the kernel that starts the step
// (OV_OPT_HOLECUT_LIST); nmc = 0: none.
struct MaskJob {
  const double* poses;
  const double4* spheres;
  const int4* tile_info;
  unsigned long long* sub_mask;
  int32_t* mask_counts;
  long long nsub, nmc;
  int ngrids;
};

// The mask chunks go to the blocks from the last one down, so that where the
// start kernel has fewer tiles to reset than blocks, different blocks take
// the two jobs.
__device__ __forceinline__ void mask_job(const MaskJob& mj, const GridDev* __restrict__ grids) {
  __shared__ MaskLds ML;
  mask_stage(ML, grids, mj.ngrids, mj.poses);
  mask_chunks(ML, mj.spheres, mj.tile_info, mj.nsub, mj.sub_mask, mj.mask_counts, mj.nmc,
              (long long)gridDim.x - 1 - blockIdx.x, gridDim.x);
}

// The culled hole cut runs in two kernels, in stream order:
//  k_fill_masks      every node's flag as if no blank region reached it
//                    (field, or fringe on the fixed outer-boundary layers),
//                    and in other blocks of the same launch which blank
//                    regions may reach each sub-tile, listing the sub-tiles
//                    with any (the candidates);
//  k_holecut_cand_*  the candidate sub-tiles' nodes tested, their flags
//                    rewritten, and the tiles within buffer reach of a hole
//                    put on the near list for the fringe pass.
// The fill is a pure stream over the flag array in whole 16-byte words, 4
// per thread per iteration, a block's words contiguous: zeros over grids
// without outer layers, a copy of the base flags (computed once) over grids
// with them. The partial words at a range's ends are written bytewise by
// one thread each.
constexpr int kFillUnroll = 4;

__device__ __forceinline__ void flag_fill_body(uint8_t* __restrict__ flags, const uint8_t* __restrict__ base,
                                               const long long* __restrict__ fill_ranges, int nranges,
                                               long long fill_words, long long bid, long long nblocks) {
  gmem<long long>* R = gp(fill_ranges);
  const long long nthreads = nblocks * blockDim.x;
  for (long long w0 = bid * blockDim.x * kFillUnroll + threadIdx.x; w0 < fill_words;
       w0 += nthreads * kFillUnroll) {
#pragma unroll
    for (int q = 0; q < kFillUnroll; ++q) {
      const long long w = w0 + (long long)q * blockDim.x;
      if (w >= fill_words) break;
      int r = 0;
      while (r + 1 < nranges && R[4 * (r + 1) + 2] <= w) ++r;
      const long long x = 16 * ((R[4 * r] + 15) / 16 + w - R[4 * r + 2]);  // byte offset of the word
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (R[4 * r + 3]) v = *reinterpret_cast<const uint4*>(base + x);
      *reinterpret_cast<uint4*>(flags + x) = v;
    }
  }
  if (bid == 0 && (int)threadIdx.x < nranges) {
    // bytes before the first and after the last whole word of range r
    const long long a = R[4 * threadIdx.x], b = R[4 * threadIdx.x + 1];
    const bool copy = R[4 * threadIdx.x + 3] != 0;
    const long long wa = 16 * ((a + 15) / 16), wb = 16 * (b / 16);
    const long long head_end = min(wa, b), tail_begin = max(wb, head_end);  // at most 15 bytes each
    for (long long x = a; x < head_end; ++x) flags[x] = copy ? base[x] : (uint8_t)OV_STATE_FIELD;
    for (long long x = tail_begin; x < b; ++x) flags[x] = copy ? base[x] : (uint8_t)OV_STATE_FIELD;
  }
}

// Block 0 also starts the step (new stamp, empty lists).
// The step executors' start of a step on a flags buffer that holds the
// previous step of its slot: every byte that step changed from the base
// flags (holes, buffer layers) lies in a tile of its near list (a hole's own
// tile is on it, and buffer layers are only written in listed tiles), so
// only those tiles are returned to their base flags (a copy, or field for a
// grid without outer layers): one workgroup per tile, a quarter row of 16
// bytes per thread. Also starts the step as k_flag_fill does.
__global__ void __launch_bounds__(256) k_flag_reset(const GridDev* __restrict__ grids, uint8_t* __restrict__ flags,
                                                   const uint8_t* __restrict__ base,
                                                   const int4* __restrict__ old_list,
                                                   const int32_t* __restrict__ old_count, unsigned int stamp,
                                                   unsigned int* __restrict__ counter,
                                                   unsigned int* __restrict__ d_stamp,
                                                   int32_t* __restrict__ near_count,
                                                   int32_t* __restrict__ chunk_list_count,
                                                   int32_t* __restrict__ super_counts, long long n_super_counts,
                                                   unsigned long long* __restrict__ stats, MaskJob mj) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    k_begin_step_body(stamp, counter, d_stamp, near_count, chunk_list_count);
    atomicAdd(&stat_slot(stats)[OV_STAT_FLAG_STARTS], 1ULL);
  }
  if (mj.nmc > 0) mask_job(mj, grids);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_super_counts;
       i += (long long)gridDim.x * blockDim.x)
    super_counts[i] = 0;
  const int n = *old_count;
  unsigned int written = 0, base_read = 0;  // this thread's bytes (work counters)
  static_assert(kTileI == 64 && kTileJ * kTileK * 4 == 256, "a 256-thread block covers a tile, 16 bytes a thread");
  for (int idx = blockIdx.x; idx < n; idx += gridDim.x) {
    const int4 info = old_list[idx];
    const GridDev& G = grids[info.x];
    const int row = threadIdx.x >> 2, q = threadIdx.x & 3;
    const int j = info.z * kTileJ + (row & 7), k = info.w * kTileK + (row >> 3);
    if (j >= G.nj || k >= G.nk) continue;
    const int i0 = info.y * kTileI + 16 * q, i1 = min(G.ni, i0 + 16);
    const long long r = G.node_off + (long long)G.ni * ((long long)j + (long long)G.nj * k);
    uint8_t* dst = flags + r + i0;
    if (i1 > i0) {
      written += (unsigned int)(i1 - i0);
      if (G.has_outer) base_read += (unsigned int)(i1 - i0);
    }
    if (i1 - i0 == 16 && ((((uintptr_t)dst) | ((uintptr_t)(base + r + i0))) & 15) == 0) {
      // a whole aligned 16-byte run: one vector store (base flags share the layout)
      constexpr uint32_t fw = 0x01010101u * (uint32_t)OV_STATE_FIELD;
      *reinterpret_cast<uint4*>(dst) =
          G.has_outer ? *reinterpret_cast<const uint4*>(base + r + i0) : make_uint4(fw, fw, fw, fw);
    } else {
      for (int i = i0; i < i1; ++i) flags[r + i] = G.has_outer ? base[r + i] : (uint8_t)OV_STATE_FIELD;
    }
  }
  // the wavefront's bytes, summed with shuffles, one atomic per counter
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    written += __shfl_xor(written, o, 64);
    base_read += __shfl_xor(base_read, o, 64);
  }
  if ((threadIdx.x & 63) == 0 && written) {
    unsigned long long* slot = stat_slot(stats);
    atomicAdd(&slot[OV_STAT_FLAG_BYTES_WRITTEN], (unsigned long long)written);
    if (base_read) atomicAdd(&slot[OV_STAT_BASE_BYTES_READ], (unsigned long long)base_read);
  }
}

__global__ void __launch_bounds__(256) k_flag_fill(const GridDev* __restrict__ grids, uint8_t* __restrict__ flags,
                                                  const uint8_t* __restrict__ base,
                                                  const long long* __restrict__ fill_ranges, int nranges,
                                                  long long fill_words, unsigned int stamp,
                                                  unsigned int* __restrict__ counter,
                                                  unsigned int* __restrict__ d_stamp,
                                                  int32_t* __restrict__ near_count,
                                                  int32_t* __restrict__ chunk_list_count,
                                                  int32_t* __restrict__ super_counts, long long n_super_counts,
                                                  unsigned long long* __restrict__ stats, long long nodes,
                                                  long long base_nodes, MaskJob mj) {
  if (mj.nmc > 0) mask_job(mj, grids);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    k_begin_step_body(stamp, counter, d_stamp, near_count, chunk_list_count);
    unsigned long long* slot = stat_slot(stats);
    atomicAdd(&slot[OV_STAT_FLAG_STARTS], 1ULL);
    atomicAdd(&slot[OV_STAT_FLAG_BYTES_WRITTEN], (unsigned long long)nodes);
    atomicAdd(&slot[OV_STAT_BASE_BYTES_READ], (unsigned long long)base_nodes);
  }
  // the slot's superchunk counts start from zero (the last reader of this
  // slot's counts, the previous compaction using it, is done)
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_super_counts;
       i += (long long)gridDim.x * blockDim.x)
    super_counts[i] = 0;
  flag_fill_body(flags, base, fill_ranges, nranges, fill_words, blockIdx.x, gridDim.x);
}

// Candidate sub-tiles (kSubI x kTileJ x kTileK nodes), one block each at a
// time (the variant for few candidates: shortest latency per sub-tile):
// thread t takes the 4 nodes i0 + 4 (t % 4) .. + 3 of row
// (j0 + (t / 4) % 8, k0 + t / 32), loads their coordinates at once, tests
// them against the blank regions of the sub-tile's mask only and writes
// their 4 flags.
static_assert(kSubI == 16 && kTileJ * kTileK * 4 == 256, "a 256-thread block covers a sub-tile with 4 nodes each");

template <typename CT, bool MESH>
__device__ __forceinline__ void cand_block(const HoleLds& L, const TileGeo* TG, const GridDev* __restrict__ grids,
                                           uint8_t* __restrict__ flags, const int4 ti, int sub,
                                           unsigned long long mask, unsigned int stamp, unsigned int* __restrict__ tile_near,
                                           int4* __restrict__ near_list, int32_t* __restrict__ near_count,
                                           unsigned int* __restrict__ tile_hole, unsigned long long* __restrict__ stats) {
  const int A = uniform_i32(ti.x);
  const TileGeo& G = TG[A];
  const int ni = G.ni, nj = G.nj, nk = G.nk;
  const int o0 = G.o[0], o1 = G.o[1], o2 = G.o[2], o3 = G.o[3], o4 = G.o[4], o5 = G.o[5];
  const int t = threadIdx.x;
  const int i = ti.y * kTileI + (sub % kSubPerTile) * kSubI + 4 * (t & 3), j = ti.z * kTileJ + ((t >> 2) & 7),
            k = ti.w * kTileK + (t >> 5);
  const bool ok = i < ni && j < nj && k < nk;
  const int n = ok ? min(4, ni - i) : 0;
  const bool outer = L.outer[A] != 0;
  const bool row_outer = outer && (j < o2 || j >= nj - o3 || k < o4 || k >= nk - o5);
  bool hole = false;
  unsigned int hm = 0u;  // bit r: node i + r is a hole
  if constexpr (!MESH) {
    if (ok) {
      const int m0 = i + ni * (j + nj * k);  // node index in grid A (< 2^31)
      uint8_t* dst = flags + L.off[A] + m0;
      gmem<CT>* Xa = gp((const CT*)L.X[A]) + m0;
      gmem<CT>* Ya = gp((const CT*)L.Y[A]) + m0;
      gmem<CT>* Za = gp((const CT*)L.Z[A]) + m0;
      CT X[4], Y[4], Z[4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (r < n) {
          X[r] = Xa[r];
          Y[r] = Ya[r];
          Z[r] = Za[r];
        }
      uint32_t word = 0u;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r >= n) continue;
        const int cause = holecut_node<CT, false>(L, grids, A, m0 + r, X[r], Y[r], Z[r], mask);
        uint32_t f = OV_STATE_FIELD;
        if (cause >= 0) {
          f = kHole | (cause << 2);
          hole = true;
          hm |= 1u << r;
        } else if (outer && (row_outer || i + r < o0 || i + r >= ni - o1)) {
          f = kFringe | (OV_CAUSE_BOUNDARY << 2);
        }
        word |= f << (8 * r);
      }
      if (n == 4 && (((uintptr_t)dst) & 3) == 0) {
        *reinterpret_cast<uint32_t*>(dst) = word;
      } else {
        for (int e = 0; e < n; ++e) dst[e] = (uint8_t)(word >> (8 * e));
      }
    }
  } else {
    const int m0 = i + ni * (j + nj * k);  // node index in grid A (< 2^31)
    int cz[4] = {-1, -1, -1, -1};
    if (ok) {
      gmem<CT>* Xa = gp((const CT*)L.X[A]) + m0;
      gmem<CT>* Ya = gp((const CT*)L.Y[A]) + m0;
      gmem<CT>* Za = gp((const CT*)L.Z[A]) + m0;
      CT X[4], Y[4], Z[4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (r < n) {
          X[r] = Xa[r];
          Y[r] = Ya[r];
          Z[r] = Za[r];
        }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (r < n) cz[r] = holecut_node<CT, MESH, MESH>(L, grids, A, m0 + r, X[r], Y[r], Z[r], mask);
    }
    if constexpr (MESH) {
      // nodes near a triangulated surface cluster in a few lanes: their parity
      // tests are shared out over the whole workgroup, one node per thread
      __shared__ int dq_node[1024];
      __shared__ int dq_res[1024];
      __shared__ int dq_n;
      bool deferred = false;
#pragma unroll
      for (int r = 0; r < 4; ++r) deferred |= cz[r] == kDeferNode;
      if (t == 0) dq_n = 0;
      if (__syncthreads_or(deferred)) {  // (most candidate sub-tiles have none)
        int slot[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (cz[r] == kDeferNode) {
            slot[r] = atomicAdd(&dq_n, 1);
            dq_node[slot[r]] = m0 + r;
          }
        __syncthreads();
        const int qn = dq_n;
        for (int q = t; q < qn; q += blockDim.x)
          dq_res[q] = holecut_node_exact<MESH>(L, grids, A, dq_node[q], mask);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (cz[r] == kDeferNode) cz[r] = dq_res[slot[r]];
      }
    }
    if (ok) {
      uint8_t* dst = flags + L.off[A] + m0;
      uint32_t word = 0u;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r >= n) continue;
        const int cause = cz[r];
        uint32_t f = OV_STATE_FIELD;
        if (cause >= 0) {
          f = kHole | (cause << 2);
          hole = true;
          hm |= 1u << r;
        } else if (outer && (row_outer || i + r < o0 || i + r >= ni - o1)) {
          f = kFringe | (OV_CAUSE_BOUNDARY << 2);
        }
        word |= f << (8 * r);
      }
      if (n == 4 && (((uintptr_t)dst) & 3) == 0) {
        *reinterpret_cast<uint32_t*>(dst) = word;
      } else {
        for (int e = 0; e < n; ++e) dst[e] = (uint8_t)(word >> (8 * e));
      }
    }
  }
  int nr = n;
  for (int o = 32; o > 0; o >>= 1) nr += __shfl_xor(nr, o, 64);
  if ((t & 63) == 0) atomicAdd(&stat_slot(stats)[OV_STAT_HOLECUT_NODES_READ], (unsigned long long)nr);
  // the box of the sub-tile's holes: per wavefront, then over the block
  __shared__ int wbox[4][6];
  HoleBox hb;
  hb.lo[0] = hm ? i + __builtin_ctz(hm) : INT_MAX;
  hb.hi[0] = hm ? i + 31 - __builtin_clz(hm) : INT_MIN;
  hb.lo[1] = hm ? j : INT_MAX;
  hb.hi[1] = hm ? j : INT_MIN;
  hb.lo[2] = hm ? k : INT_MAX;
  hb.hi[2] = hm ? k : INT_MIN;
  if (__any(hm != 0u)) hole_box_wave(hb);
  if ((t & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      wbox[t >> 6][d] = hb.lo[d];
      wbox[t >> 6][3 + d] = hb.hi[d];
    }
  }
  if (__syncthreads_or(hole)) {  // (the same in every thread)
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        hb.lo[d] = min(hb.lo[d], wbox[w][d]);
        hb.hi[d] = max(hb.hi[d], wbox[w][3 + d]);
      }
    __syncthreads();  // every thread has read the boxes before the next candidate writes them
    mark_near_box(hb, t, 256, ti.x, ni, nj, nk, G.per, G.tiles_i, G.tiles_j, G.tile_off, stamp, tile_near, near_list,
                  near_count);
    if (t == 0) tile_hole[sub / kSubPerTile] = stamp;  // this step has a hole in the tile
  }
}

// Candidate sub-tiles, one wavefront each at a time (the variant for many
// candidates: no block barrier per sub-tile, the block's wavefronts on
// different candidates at once): lane l takes the 16 nodes i0 .. i0 + 15 of
// row (j0 + l % 8, k0 + l / 8), loads all their coordinates (FP32; FP64 in
// two halves) before testing any, tests them against the blank regions of
// the sub-tile's mask only and writes their 16 flags in one store.
template <typename CT, bool MESH>
__device__ __forceinline__ void cand_wave(const HoleLds& L, const TileGeo* TG, const GridDev* __restrict__ grids,
                                          uint8_t* __restrict__ flags, const int4 ti, int sub,
                                          unsigned long long mask, unsigned int stamp, unsigned int* __restrict__ tile_near,
                                          int4* __restrict__ near_list, int32_t* __restrict__ near_count,
                                          unsigned int* __restrict__ tile_hole, unsigned long long* __restrict__ stats) {
  constexpr int kBatch = sizeof(CT) == 4 ? kSubI : kSubI / 2;  // nodes whose coordinates are loaded together
  const int lane = threadIdx.x & 63;
  const int A = uniform_i32(ti.x);
  const TileGeo& G = TG[A];
  const int ni = G.ni, nj = G.nj, nk = G.nk;
  const int o0 = G.o[0], o1 = G.o[1], o2 = G.o[2], o3 = G.o[3], o4 = G.o[4], o5 = G.o[5];
  const int i = ti.y * kTileI + (sub % kSubPerTile) * kSubI, j = ti.z * kTileJ + (lane & 7),
            k = ti.w * kTileK + (lane >> 3);
  const bool ok = i < ni && j < nj && k < nk;
  const int n = ok ? min(kSubI, ni - i) : 0;
  const bool outer = L.outer[A] != 0;
  const bool row_outer = outer && (j < o2 || j >= nj - o3 || k < o4 || k >= nk - o5);
  bool hole = false;
  unsigned int hm = 0u;  // bit e: node i + e is a hole
  if (ok) {
    const int m0 = i + ni * (j + nj * k);  // node index in grid A (< 2^31)
    uint8_t* dst = flags + L.off[A] + m0;
    gmem<CT>* Xa = gp((const CT*)L.X[A]) + m0;
    gmem<CT>* Ya = gp((const CT*)L.Y[A]) + m0;
    gmem<CT>* Za = gp((const CT*)L.Z[A]) + m0;
    uint32_t w[4] = {0u, 0u, 0u, 0u};  // the 16 flag bytes
#pragma unroll
    for (int b0 = 0; b0 < kSubI; b0 += kBatch) {
      CT X[kBatch], Y[kBatch], Z[kBatch];
      // every load of the batch issued before the first test (a node past
      // the row's end re-reads its last node and is not tested)
#pragma unroll
      for (int r = 0; r < kBatch; ++r) {
        const int e = min(b0 + r, n - 1);
        X[r] = Xa[e];
        Y[r] = Ya[e];
        Z[r] = Za[e];
      }
#pragma unroll
      for (int r = 0; r < kBatch; ++r) {
        const int e = b0 + r;
        if (e >= n) continue;
        const int cause = holecut_node<CT, MESH>(L, grids, A, m0 + e, X[r], Y[r], Z[r], mask);
        uint32_t f = OV_STATE_FIELD;
        if (cause >= 0) {
          f = kHole | (cause << 2);
          hole = true;
          hm |= 1u << e;
        } else if (outer && (row_outer || i + e < o0 || i + e >= ni - o1)) {
          f = kFringe | (OV_CAUSE_BOUNDARY << 2);
        }
        w[e >> 2] |= f << (8 * (e & 3));
      }
    }
    if (n == 16 && (((uintptr_t)dst) & 15) == 0) {
      *reinterpret_cast<uint4*>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
      for (int e = 0; e < n; ++e) {
        const uint32_t wd = e < 4 ? w[0] : e < 8 ? w[1] : e < 12 ? w[2] : w[3];
        dst[e] = (uint8_t)(wd >> (8 * (e & 3)));
      }
    }
  }
  int nr = n;
  for (int o = 32; o > 0; o >>= 1) nr += __shfl_xor(nr, o, 64);
  if (lane == 0) atomicAdd(&stat_slot(stats)[OV_STAT_HOLECUT_NODES_READ], (unsigned long long)nr);
  if (__any(hole)) {
    HoleBox hb;
    hb.lo[0] = hm ? i + __builtin_ctz(hm) : INT_MAX;
    hb.hi[0] = hm ? i + 31 - __builtin_clz(hm) : INT_MIN;
    hb.lo[1] = hm ? j : INT_MAX;
    hb.hi[1] = hm ? j : INT_MIN;
    hb.lo[2] = hm ? k : INT_MAX;
    hb.hi[2] = hm ? k : INT_MIN;
    hole_box_wave(hb);
    mark_near_box(hb, lane, 64, ti.x, ni, nj, nk, G.per, G.tiles_i, G.tiles_j, G.tile_off, stamp, tile_near,
                  near_list, near_count);
    if (lane == 0) tile_hole[sub / kSubPerTile] = stamp;  // this step has a hole in the tile
  }
}

// The culled hole cut after the fill: each block takes an interleaved share
// of the sub-tiles (sub-tile s goes to block s mod gridDim, so neighbouring
// sub-tiles, which are the ones near a body, spread over the blocks), 256
// per round. One thread per sub-tile computes its mask; the sub-tiles with
// any (the candidates) are listed in LDS, and the block then tests their
// nodes, one candidate per block (cand_block) or per wavefront (cand_wave)
// at a time. No list leaves the block, so nothing needs resetting between
// steps.
template <typename CT, bool WAVE, bool MESH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MESH ? 1 : (sizeof(CT) == 4 ? 4 : 3)))) k_holecut_sub(const GridDev* __restrict__ grids, int ngrids,
                                                    const double* __restrict__ poses, uint8_t* __restrict__ flags,
                                                    const double4* __restrict__ spheres,
                                                    const int4* __restrict__ tile_info, long long nsub,
                                                    long long perm,
                                                    const unsigned int* __restrict__ d_stamp,
                                                    unsigned int* __restrict__ tile_near,
                                                    int4* __restrict__ near_list,
                                                    int32_t* __restrict__ near_count,
                                                    unsigned int* __restrict__ tile_hole,
                                                    unsigned long long* __restrict__ stats) {
  __shared__ HoleLds L;
  __shared__ TileGeo TG[kMaxGrids];
  __shared__ int c_sub[256];
  __shared__ unsigned long long c_mask[256];
  __shared__ int4 c_info[256];
  __shared__ int c_n;
  stage_tile_geo(TG, grids, ngrids);
  holecut_stage<CT>(L, grids, ngrids, poses);  // ends with a barrier
  const unsigned int stamp = *d_stamp;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&stat_slot(stats)[OV_STAT_HOLECUT_CALLS], 1ULL);
  const long long nb = gridDim.x;
  for (long long r0 = 0; r0 < nsub; r0 += 256 * nb) {
    if (threadIdx.x == 0) c_n = 0;
    __syncthreads();
    // position idx of the round visits sub-tile idx * perm mod nsub (perm is
    // prime to nsub: a bijection), which scatters the sub-tiles of one body's
    // neighbourhood over the blocks; a plain stride would fold a grid's
    // planes of sub-tiles onto the same blocks whenever the plane length is a
    // multiple of the block count
    const long long idx = r0 + (long long)threadIdx.x * nb + blockIdx.x;
    const long long sub = idx < nsub ? (idx * perm) % nsub : nsub;
    if (sub < nsub) {
      const int4 info = tile_info[sub / kSubPerTile];
      const unsigned long long m = sub_mask(L, info.x, spheres[sub]);
      if (m) {
        const int slot = atomicAdd(&c_n, 1);
        c_sub[slot] = (int)sub;
        c_mask[slot] = m;
        c_info[slot] = info;
      }
    }
    __syncthreads();
    const int n = c_n;
    if (WAVE) {
      for (int c = threadIdx.x >> 6; c < n; c += 4)
        cand_wave<CT, MESH>(L, TG, grids, flags, c_info[c], uniform_i32(c_sub[c]), uniform_u64(c_mask[c]), stamp,
                            tile_near, near_list, near_count, tile_hole, stats);
    } else {
      for (int c = 0; c < n; ++c)
        cand_block<CT, MESH>(L, TG, grids, flags, c_info[c], c_sub[c], uniform_u64(c_mask[c]), stamp, tile_near,
                             near_list, near_count, tile_hole, stats);
    }
    __syncthreads();  // the list is rebuilt by the next round
  }
}

// The culled hole cut after a start kernel that culled the sub-tiles
// (OV_OPT_HOLECUT_LIST): the step's candidates, in ascending sub-tile order,
// are ranked from the start kernel's per-chunk counts, and block b tests
// candidates b, b + gridDim, ... (one each when there are fewer candidates
// than blocks). Every block scans the chunk counts itself, 1024 chunks at a
// time (4 per thread), finds the chunk of each of its ranks by bisection of
// the scanned counts, and the candidate in the chunk by the rank of its
// non-zero mask among the chunk's.
template <typename CT, bool MESH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MESH ? 1 : 4)))
    k_holecut_list(const GridDev* __restrict__ grids, int ngrids, const double* __restrict__ poses,
                   uint8_t* __restrict__ flags, const int4* __restrict__ tile_info,
                   const unsigned long long* __restrict__ sub_masks, const int32_t* __restrict__ mask_counts,
                   long long nsub, long long nmc, const unsigned int* __restrict__ d_stamp,
                   unsigned int* __restrict__ tile_near, int4* __restrict__ near_list,
                   int32_t* __restrict__ near_count, unsigned int* __restrict__ tile_hole,
                   unsigned long long* __restrict__ stats) {
  static_assert(kMaskChunk == 256, "one sub-tile of a chunk per thread");
  constexpr int kBatch = 4 * 256;  // chunks scanned per round
  __shared__ HoleLds L;
  __shared__ TileGeo TG[kMaxGrids];
  __shared__ int pre[kBatch + 1];  // exclusive prefix of the round's chunk counts; [kBatch] their sum
  __shared__ int wsum[4];
  __shared__ int c_sub;
  __shared__ unsigned long long c_mask;
  __shared__ int4 c_info;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // the first round's counts are loaded before the staging's barriers
  int v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = 4 * t + e < nmc ? mask_counts[4 * t + e] : 0;
  stage_tile_geo(TG, grids, ngrids);
  holecut_stage<CT>(L, grids, ngrids, poses);  // ends with a barrier
  const unsigned int stamp = *d_stamp;
  if (blockIdx.x == 0 && t == 0) atomicAdd(&stat_slot(stats)[OV_STAT_HOLECUT_CALLS], 1ULL);
  long long before = 0;         // candidates in the chunks of the earlier rounds
  long long r = blockIdx.x;     // this block's next rank
  for (long long c0 = 0; c0 < nmc; c0 += kBatch) {
    if (c0 > 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = c0 + 4 * t + e < nmc ? mask_counts[c0 + 4 * t + e] : 0;
    }
    // block-wide exclusive scan of the threads' sums
    const int mine = v[0] + v[1] + v[2] + v[3];
    int inc = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int ex = inc - mine;
    for (int w = 0; w < wv; ++w) ex += wsum[w];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    pre[4 * t] = ex;
    pre[4 * t + 1] = ex + v[0];
    pre[4 * t + 2] = ex + v[0] + v[1];
    pre[4 * t + 3] = ex + v[0] + v[1] + v[2];
    if (t == 0) pre[kBatch] = total;
    __syncthreads();
    while (r < before + total) {  // (the same in every thread)
      const int k = (int)(r - before);
      // the chunk of rank k: the last e with pre[e] <= k (its count is > 0)
      int lo = 0, hi = kBatch - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= k) lo = mid;
        else hi = mid - 1;
      }
      const int kk = k - pre[lo];
      const long long sub = (c0 + lo) * kMaskChunk + t;
      unsigned long long m = 0;
      int4 info = make_int4(0, 0, 0, 0);
      if (sub < nsub) {
        m = sub_masks[sub];
        info = tile_info[sub / kSubPerTile];
      }
      const unsigned long long bm = __ballot(m != 0ull);
      if (lane == 0) wsum[wv] = (int)__popcll(bm);
      __syncthreads();
      int rank = (int)__popcll(bm & ((1ull << lane) - 1ull));
      for (int w = 0; w < wv; ++w) rank += wsum[w];
      if (m != 0ull && rank == kk) {
        c_sub = (int)sub;
        c_mask = m;
        c_info = info;
      }
      __syncthreads();
      cand_block<CT, MESH>(L, TG, grids, flags, c_info, c_sub, uniform_u64(c_mask), stamp, tile_near, near_list,
                           near_count, tile_hole, stats);
      __syncthreads();  // c_sub, c_mask, c_info and wsum are rewritten next
      r += gridDim.x;
    }
    before += total;
  }
}

// Near list from the streaming hole cut's per-tile hole stamps: one thread per
// tile; a tile holding a hole lists its 125 reach combinations.
__global__ void __launch_bounds__(256) k_near_from_holes(const GridDev* __restrict__ grids,
                                                        const unsigned int* __restrict__ tile_hole,
                                                        const int4* __restrict__ tile_info, long long total_tiles,
                                                        const unsigned int* __restrict__ d_stamp,
                                                        unsigned int* __restrict__ tile_near,
                                                        int4* __restrict__ near_list,
                                                        int32_t* __restrict__ near_count) {
  const unsigned int stamp = *d_stamp;
  for (long long tile = (long long)blockIdx.x * blockDim.x + threadIdx.x; tile < total_tiles;
       tile += (long long)gridDim.x * blockDim.x) {
    if (tile_hole[tile] != stamp) continue;
    const int4 info = tile_info[tile];
    const GeomR G(grids[info.x]);
    const int ti = info.y, tj = info.z, tk = info.w;
    for (int e = 0; e < 125; ++e)
      mark_near(e, info.x, ti, tj, tk, G.ni, G.nj, G.nk, G.per, G.tiles_i, G.tiles_j, G.tile_off, stamp, tile_near, near_list,
                near_count);
  }
}

// Near list from a flags buffer alone (the fringe call of the C ABI, which
// may be given flags from any hole cut): one block per tile at a time, a
// quarter row of 16 flag bytes per thread; a tile holding a hole lists its
// 125 reach combinations, one per thread.
__global__ void __launch_bounds__(256) k_near_from_flags(const GridDev* __restrict__ grids,
                                                        const uint8_t* __restrict__ flags,
                                                        const int4* __restrict__ tile_info, long long total_tiles,
                                                        const unsigned int* __restrict__ d_stamp,
                                                        unsigned int* __restrict__ tile_near,
                                                        int4* __restrict__ near_list,
                                                        int32_t* __restrict__ near_count) {
  static_assert(kTileI == 64 && kTileJ * kTileK * 4 == 256, "a 256-thread block covers a tile, 16 bytes a thread");
  const unsigned int stamp = *d_stamp;
  for (long long tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    const int4 info = tile_info[tile];
    const GridDev& G = grids[info.x];
    const int row = threadIdx.x >> 2, q = threadIdx.x & 3;
    const int j = info.z * kTileJ + (row & 7), k = info.w * kTileK + (row >> 3);
    bool hole = false;
    if (j < G.nj && k < G.nk) {
      const int i0 = info.y * kTileI + 16 * q, i1 = min(G.ni, i0 + 16);
      const uint8_t* p = flags + G.node_off + (long long)G.ni * ((long long)j + (long long)G.nj * k);
      if (i1 - i0 == 16 && (((uintptr_t)(p + i0)) & 15) == 0) {
        const uint4 v = *reinterpret_cast<const uint4*>(p + i0);
        // state bits 0-1 of each byte equal to 1 (HOLE): bit 0 set, bit 1 clear
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) hole |= ((w[e] & ~(w[e] >> 1)) & 0x01010101u) != 0u;
      } else {
        for (int i = i0; i < i1; ++i) hole |= (p[i] & 3) == kHole;
      }
    }
    hole = __syncthreads_or(hole);
    if (hole && threadIdx.x < 125)
      mark_near((int)threadIdx.x, info.x, info.y, info.z, info.w, G.ni, G.nj, G.nk, G.per, G.tiles_i, G.tiles_j,
                G.tile_off, stamp, tile_near, near_list, near_count);
  }
}

FrontScratch ctx_scratch(ov_ctx* ctx, int slot, int gen) {
  const long long nt = std::max(1LL, ctx->total_tiles);
  FrontScratch f;
  f.counter = ctx->d_stamp;
  f.stamp = ctx->d_stamp + 1 + slot;
  f.near_list = ctx->d_near_list + (gen * kSlots + slot) * nt;
  f.near_count = ctx->d_near_count + gen * kSlots + slot;
  f.tile_near = ctx->d_tile_near + (long long)slot * nt;
  f.chunk_stamp = ctx->d_chunk_stamp + (long long)slot * ctx->nchunks;
  f.chunk_list = ctx->d_chunk_list + (long long)slot * ctx->nchunks;
  f.chunk_list_count = ctx->d_chunk_list_count + slot;
  f.chunk_counts = ctx->d_chunk_counts + (long long)slot * ctx->nchunks;
  f.super_counts = ctx->d_super_counts + (long long)slot * kSuperSlots * ctx->nsuper;
  f.super_offsets = ctx->d_super_offsets + (long long)slot * (ctx->nsuper + 1);
  return f;
}

hipError_t launch_near_list_in(ov_ctx* ctx, const uint8_t* flags, hipStream_t s, const FrontScratch& fs) {
  const long long nt = ctx->total_tiles;
  const long long nb = std::max(1LL, std::min(nt, (long long)ctx->num_cus * 8));
  hipLaunchKernelGGL(k_near_from_flags, dim3((unsigned)nb), dim3(256), 0, s, ctx->d_grids, flags, ctx->d_tile_info,
                     nt, fs.stamp, fs.tile_near, fs.near_list, fs.near_count);
  return hipGetLastError();
}

hipError_t launch_near_from_flags(ov_ctx* ctx, const uint8_t* flags, hipStream_t s) {
  FrontScratch fs = ctx_scratch(ctx, 0, 0);
  fs.counter = ctx->d_stamp + 1 + kSlots;  // the fringe call's own counter
  const long long nsc = kSuperSlots * ctx->nsuper;
  // a new stamp (empty near and chunk lists, zero superchunk counts)
  hipLaunchKernelGGL(k_begin_step, dim3((unsigned)std::max(1LL, std::min(64LL, (nsc + 255) / 256))), dim3(256), 0, s,
                     0u, fs.counter, fs.stamp, fs.near_count, fs.chunk_list_count, fs.super_counts, nsc, kStampHigh);
  return launch_near_list_in(ctx, flags, s, fs);
}

template <typename CT>
static void launch_holecut_t(ov_ctx* ctx, const double* poses, uint8_t* flags, hipStream_t s, unsigned int* st,
                             unsigned int* tile_hole) {
  int block = ctx->holecut_block;
  int R = ctx->holecut_npt;  // 16-byte vectors per lane per chunk
  long long span = (long long)block * Vec16<CT>::W * R;
  long long chunks = 0;
  for (auto& g : ctx->grids) chunks += (g.d.nnodes + span - 1) / span;
  int per_cu = ctx->persist > 0 ? ctx->persist : 16;
  long long grid = std::max(1LL, std::min(chunks, (long long)ctx->num_cus * per_cu));
  int ng = (int)ctx->grids.size();
  if (R == 4)
    hipLaunchKernelGGL((k_holecut<CT, 4>), dim3((unsigned)grid), dim3(block), 0, s, ctx->d_grids, ng, poses, flags,
                       chunks, tile_hole, st, ctx->d_stats);
  else if (R == 2)
    hipLaunchKernelGGL((k_holecut<CT, 2>), dim3((unsigned)grid), dim3(block), 0, s, ctx->d_grids, ng, poses, flags,
                       chunks, tile_hole, st, ctx->d_stats);
  else
    hipLaunchKernelGGL((k_holecut<CT, 1>), dim3((unsigned)grid), dim3(block), 0, s, ctx->d_grids, ng, poses, flags,
                       chunks, tile_hole, st, ctx->d_stats);
}

hipError_t launch_holecut(ov_ctx* ctx, const double* poses, uint8_t* flags, hipStream_t s, int slot, int gen,
                          bool reset, unsigned int stamp) {
  const int ng = (int)ctx->grids.size();
  const long long nt = ctx->total_tiles;
  unsigned int* counter = ctx->d_stamp;
  unsigned int* st = ctx->d_stamp + 1 + slot;
  unsigned int* tn = ctx->d_tile_near + (long long)slot * std::max(1LL, nt);
  int4* nl = ctx->d_near_list + (gen * kSlots + slot) * std::max(1LL, nt);
  int32_t* nc = ctx->d_near_count + gen * kSlots + slot;
  unsigned int* th = ctx->d_tile_hole + slot * std::max(1LL, nt);
  int32_t* clc = ctx->d_chunk_list_count + slot;
  const long long nsc = kSuperSlots * ctx->nsuper;
  int32_t* sc = ctx->d_super_counts + (long long)slot * nsc;
  if (ctx->cull) {
    const long long fb = std::max(1LL, std::min((ctx->fill_words + 256 * kFillUnroll - 1) / (256 * kFillUnroll),
                                                (long long)ctx->num_cus * 32));
    const long long nsub = nt * kSubPerTile;
    MaskJob mj{};
    if (ctx->holecut_list) {
      mj.poses = poses;
      mj.spheres = (const double4*)ctx->d_tile_sphere;
      mj.tile_info = ctx->d_tile_info;
      mj.sub_mask = ctx->d_sub_mask + (long long)slot * nsub;
      mj.mask_counts = ctx->d_mask_counts + (long long)slot * ctx->nmask_chunks;
      mj.nsub = nsub;
      mj.nmc = ctx->nmask_chunks;
      mj.ngrids = ng;
    }
    if (reset) {
      const int og = 1 - gen;
      const long long rb = std::max(1LL, std::min(std::max(nt, mj.nmc), (long long)ctx->num_cus * 8));
      hipLaunchKernelGGL(k_flag_reset, dim3((unsigned)rb), dim3(256), 0, s, ctx->d_grids, flags, ctx->d_base_flags,
                         ctx->d_near_list + (og * kSlots + slot) * std::max(1LL, nt),
                         ctx->d_near_count + og * kSlots + slot, stamp, counter, st, nc, clc, sc, nsc, ctx->d_stats,
                         mj);
    } else {
      long long base_nodes = 0;
      for (const auto& g : ctx->grids)
        if (g.d.has_outer) base_nodes += g.d.nnodes;
      hipLaunchKernelGGL(k_flag_fill, dim3((unsigned)fb), dim3(256), 0, s, ctx->d_grids, flags, ctx->d_base_flags,
                         ctx->d_fill_ranges, ctx->n_fill_ranges, ctx->fill_words, stamp, counter, st, nc, clc, sc,
                         nsc,
                         ctx->d_stats, ctx->node_off.back(), base_nodes, mj);
    }
    const int per_cu = ctx->persist > 0 ? ctx->persist : 8;
    if (ctx->holecut_list) {
      const long long lb = std::max(1LL, std::min(nsub, (long long)ctx->num_cus * per_cu));
      const dim3 g((unsigned)lb), b(256);
#define OV_LIST_ARGS                                                                                             \
  ctx->d_grids, ng, poses, flags, ctx->d_tile_info, (const unsigned long long*)mj.sub_mask,                          \
      (const int32_t*)mj.mask_counts, nsub, mj.nmc, st, tn, nl, nc, th, ctx->d_stats
      const bool mixed = ctx->precision == OV_MIXED;
      if (ctx->has_mesh) {
        if (mixed) hipLaunchKernelGGL((k_holecut_list<float, true>), g, b, 0, s, OV_LIST_ARGS);
        else hipLaunchKernelGGL((k_holecut_list<double, true>), g, b, 0, s, OV_LIST_ARGS);
      } else {
        if (mixed) hipLaunchKernelGGL((k_holecut_list<float, false>), g, b, 0, s, OV_LIST_ARGS);
        else hipLaunchKernelGGL((k_holecut_list<double, false>), g, b, 0, s, OV_LIST_ARGS);
      }
#undef OV_LIST_ARGS
      return hipGetLastError();
    }
    const long long cb = std::max(1LL, std::min((nsub + 15) / 16, (long long)ctx->num_cus * per_cu));
#define OV_SUB_ARGS                                                                                             \
  ctx->d_grids, ng, poses, flags, (const double4*)ctx->d_tile_sphere, ctx->d_tile_info, nsub, ctx->sub_perm, st,     \
      tn, nl, nc, th, ctx->d_stats
    const bool mixed = ctx->precision == OV_MIXED;
    const dim3 g((unsigned)cb), b(256);
#define OV_SUB(CT, W)                                                                                  \
  do {                                                                                                 \
    if (ctx->has_mesh) hipLaunchKernelGGL((k_holecut_sub<CT, W, true>), g, b, 0, s, OV_SUB_ARGS);     \
    else hipLaunchKernelGGL((k_holecut_sub<CT, W, false>), g, b, 0, s, OV_SUB_ARGS);                  \
  } while (0)
    if (ctx->holecut_npl == 4) {
      if (mixed) OV_SUB(float, false);
      else OV_SUB(double, false);
    } else {
      if (mixed) OV_SUB(float, true);
      else OV_SUB(double, true);
    }
#undef OV_SUB
#undef OV_SUB_ARGS
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_begin_step, dim3((unsigned)std::max(1LL, std::min(64LL, (nsc + 255) / 256))), dim3(256), 0, s,
                     stamp, counter, st, nc, clc, sc, nsc, 0u);
  if (ctx->precision == OV_MIXED) launch_holecut_t<float>(ctx, poses, flags, s, st, th);
  else launch_holecut_t<double>(ctx, poses, flags, s, st, th);
  long long nb = std::max(1LL, std::min((nt + 255) / 256, (long long)ctx->num_cus * 4));
  hipLaunchKernelGGL(k_near_from_holes, dim3((unsigned)nb), dim3(256), 0, s, ctx->d_grids, th,
                     ctx->d_tile_info, nt, st, tn, nl, nc);
  return hipGetLastError();
}

// ================================================================ fringe marking
// The hole cut wrote holes and the outer-boundary layers, and listed every
// tile within buffer reach of a hole (the near list). Only those tiles can
// gain buffer nodes: one block per listed tile stages the tile plus an nf
// halo in LDS as "cause if hole, 255 otherwise" and takes the lowest cause
// within Chebyshev distance nf by a separable min filter (i, then j, then
// k). Holes are never rewritten, so updating flags in place is race-free: a
// neighbour tile only reads whether a node is a hole. Each listed tile also
// puts the compaction chunks holding its nodes on this step's chunk list
// (chunks already on the static list, which hold outer-boundary nodes, are
// always counted).
__device__ __forceinline__ int wrap_or_out(int v, int n, bool periodic) {
  if (v >= 0 && v < n) return v;
  if (!periodic) return -1;
  v %= n;
  return v < 0 ? v + n : v;
}

// Byte-wise minimum of four 7-bit values per word: bit 7 of each byte of
// (a | 0x80..) - b is set exactly where a >= b (no borrow crosses a byte,
// every byte of a | 0x80.. exceeding every byte of b), which selects b there.
__device__ __forceinline__ uint32_t bytemin7(uint32_t a, uint32_t b) {
  const uint32_t ge = (((a | 0x80808080u) - b) & 0x80808080u) >> 7;
  const uint32_t m = ge * 0xFFu;
  return (b & m) | (a & ~m);
}

// Bytes d .. d+3 of the little-endian pair (lo, hi), 0 <= d <= 4.
__device__ __forceinline__ uint32_t window4(uint32_t lo, uint32_t hi, int d) {
  return d == 0 ? lo : d == 4 ? hi : __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)d);
}

template <int NF>
__global__ void __launch_bounds__(256) k_fringe_tiles(const GridDev* __restrict__ grids, int ngrids,
                                                     uint8_t* __restrict__ flags,
                                                     const int4* __restrict__ near_list,
                                                     const int32_t* __restrict__ near_count,
                                                     const unsigned int* __restrict__ d_stamp,
                                                     const uint8_t* __restrict__ chunk_static,
                                                     unsigned int* __restrict__ chunk_stamp,
                                                     int32_t* __restrict__ chunk_list,
                                                     int32_t* __restrict__ chunk_list_count, long long n_static) {
  constexpr int H = NF > 0 ? NF : 1;  // LDS sizes (unused when NF = 0)
  constexpr int EJ = kTileJ + 2 * H, EK = kTileK + 2 * H;
  constexpr int NROW = EJ * EK * 16, NHALO = EJ * EK * 2 * H;
  // staged rows: NF halo bytes, the 64 tile bytes, NF halo bytes, padded to
  // whole words; values are hole causes (< 63) or 0x7F for "no hole", so
  // that the min filter runs on 4 bytes per word (bytemin7)
  constexpr int EIW = (kTileI + 2 * H + 3) / 4;  // words per staged row
  static_assert(kTileI == 64, "16 words per tile row");
  __shared__ uint32_t a32[EK * EJ * EIW];
  __shared__ uint32_t b32[EK * EJ * 16];
  __shared__ uint32_t c32[EK * kTileJ * 16];
  uint8_t* const a8 = reinterpret_cast<uint8_t*>(a32);
  __shared__ TileGeo TG[kMaxGrids];
  __shared__ long long noffs[kMaxGrids];
  // the count, the stamp and this block's first entry are read together
  // with the grid staging (the list is allocated for every tile, and the
  // grid never has more blocks than tiles)
  const int ntl = *near_count;
  const unsigned int stamp = *d_stamp;
  const int4 first_info = near_list[blockIdx.x];
  if ((int)blockIdx.x >= ntl) return;  // no tile for this block (same in every thread)
  stage_tile_geo(TG, grids, ngrids);
  for (int g = threadIdx.x; g < ngrids; g += blockDim.x) noffs[g] = grids[g].node_off;
  __syncthreads();
  for (int idx = blockIdx.x; idx < ntl; idx += gridDim.x) {
    const int4 info = idx == (int)blockIdx.x ? first_info : near_list[idx];
    const TileGeo G = TG[info.x];
    const long long noff = noffs[info.x];
    const int i0 = info.y * kTileI, j0 = info.z * kTileJ, k0 = info.w * kTileK;
    // chunks holding this tile's nodes (one tile row (j, k) per thread of
    // the first wavefront); issued after the staging loads below, so that
    // the atomics' round trips overlap the loads'
    auto mark_chunks = [&]() {
      if (threadIdx.x < kTileJ * kTileK) {
        const int j = j0 + (threadIdx.x & 7), k = k0 + (threadIdx.x >> 3);
        if (j < G.nj && k < G.nk) {
          const long long r = noff + (long long)G.ni * ((long long)j + (long long)G.nj * k);
          const long long last = min(G.ni, i0 + kTileI) - 1;
          long long c0 = (r + i0) / kCompactChunk;
          const long long c1 = (r + last) / kCompactChunk;
          // a chunk the tile's previous row (j - 1) ends in is that row's to mark
          if ((threadIdx.x & 7) > 0 && (r - G.ni + last) / kCompactChunk == c0) ++c0;
          for (long long ch = c0; ch <= c1; ++ch)
            if (!chunk_static[ch] && atomicExch(&chunk_stamp[ch], stamp) != stamp)
              chunk_list[n_static + atomicAdd(chunk_list_count, 1)] = (int32_t)ch;
        }
      }
    };
    if (NF == 0) {
      mark_chunks();
      continue;
    }
    uint8_t* fl = flags + noff;
    // stage hole causes with halo: 16 threads per row load the 64 interior
    // bytes as words where the row is aligned and in range, the halo bytewise
    // (out-of-range bytes read as 0, a field node). Fixed trip counts: all
    // loads are issued first, then the chunk marking, then the conversions
    // and LDS stores.
    constexpr int NIT = (NROW + 255) / 256, NHIT = (NHALO + 255) / 256;
    uint32_t raw[NIT];
    uint8_t hraw[NHIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      raw[it] = 0u;
      const int e = threadIdx.x + it * 256;
      if (e >= NROW) continue;  // only the last round is partial
      const int row = e >> 4, part = e & 15;
      const int y = row % EJ, z = row / EJ;
      const int j = wrap_or_out(j0 - NF + y, G.nj, G.per & 2);
      const int k = wrap_or_out(k0 - NF + z, G.nk, G.per & 4);
      if (j >= 0 && k >= 0) {
        const uint8_t* rowp = fl + (long long)G.ni * ((long long)j + (long long)G.nj * k);
        const int i = i0 + part * 4;
        if (i + 4 <= G.ni && (((uintptr_t)(rowp + i)) & 3) == 0) {
          raw[it] = *reinterpret_cast<const uint32_t*>(rowp + i);
        } else {
          uint32_t w = 0u;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            int ii = wrap_or_out(i + q, G.ni, G.per & 1);
            if (ii >= 0) w |= (uint32_t)rowp[ii] << (8 * q);
          }
          raw[it] = w;
        }
      }
    }
#pragma unroll
    for (int it = 0; it < NHIT; ++it) {
      hraw[it] = 0;
      const int e = threadIdx.x + it * 256;
      if (e >= NHALO) continue;  // only the last round is partial
      const int h = e % (2 * H), row = e / (2 * H);  // (H = NF here: NF = 0 never gets this far)
      const int y = row % EJ, z = row / EJ;
      const int x = h < NF ? h : kTileI + h;  // NF halo bytes on each side
      const int i = wrap_or_out(i0 - NF + x, G.ni, G.per & 1);
      const int j = wrap_or_out(j0 - NF + y, G.nj, G.per & 2);
      const int k = wrap_or_out(k0 - NF + z, G.nk, G.per & 4);
      if (i >= 0 && j >= 0 && k >= 0)
        hraw[it] = fl[(long long)i + (long long)G.ni * ((long long)j + (long long)G.nj * k)];
    }
    mark_chunks();
    bool any_hole = false;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = threadIdx.x + it * 256;
      if (e >= NROW) continue;
      const int row = e >> 4, part = e & 15;
      const int y = row % EJ, z = row / EJ;
      uint8_t v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint8_t f = (uint8_t)(raw[it] >> (8 * q));
        v[q] = ((f & 3) == kHole) ? (uint8_t)(f >> 2) : (uint8_t)0x7F;
        a8[(z * EJ + y) * 4 * EIW + NF + part * 4 + q] = v[q];
      }
      any_hole |= (v[0] & v[1] & v[2] & v[3]) != 0x7F;
    }
#pragma unroll
    for (int it = 0; it < NHIT; ++it) {
      const int e = threadIdx.x + it * 256;
      if (e >= NHALO) continue;
      const int h = e % (2 * H), row = e / (2 * H);
      const int y = row % EJ, z = row / EJ;
      const int x = h < NF ? h : kTileI + h;
      const uint8_t f = hraw[it];
      const uint8_t v = ((f & 3) == kHole) ? (uint8_t)(f >> 2) : (uint8_t)0x7F;
      a8[(z * EJ + y) * 4 * EIW + x] = v;
      any_hole |= v != 0x7F;
    }
    // no hole within nf of the tile: nothing to mark (same in every thread)
    if (!__syncthreads_or(any_hole)) continue;
    // separable min filter over the (2 nf + 1)^3 box, 4 nodes per word, with
    // fixed trip counts so that each pass's LDS reads are issued together:
    // along i (windows of the staged row), along j, along k
    constexpr int N1 = EK * EJ * 16, N2 = EK * kTileJ * 16, N3 = kTileK * kTileJ * 16;
#pragma unroll
    for (int it = 0; it < (N1 + 255) / 256; ++it) {
      const int e = threadIdx.x + it * 256;
      if (e >= N1) break;
      const int row = e >> 4, w = e & 15;
      const uint32_t* r = a32 + row * EIW + w;
      const uint32_t w0 = r[0], w1 = r[1], w2 = (2 * NF > 4) ? r[2] : 0u;
      uint32_t m = w0;
#pragma unroll
      for (int d = 1; d <= 2 * NF; ++d) m = bytemin7(m, d <= 4 ? window4(w0, w1, d) : window4(w1, w2, d - 4));
      b32[e] = m;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < (N2 + 255) / 256; ++it) {
      const int e = threadIdx.x + it * 256;
      if (e >= N2) break;
      const int w = e & 15, y = (e >> 4) & 7, z = e >> 7;
      uint32_t m = b32[(z * EJ + y) * 16 + w];
#pragma unroll
      for (int d = 1; d <= 2 * NF; ++d) m = bytemin7(m, b32[(z * EJ + y + d) * 16 + w]);
      c32[e] = m;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < N3 / 256; ++it) {
      const int e = threadIdx.x + it * 256;
      const int w = e & 15, y = (e >> 4) & 7, z = e >> 7;
      uint32_t cause = c32[(z * kTileJ + y) * 16 + w];
#pragma unroll
      for (int d = 1; d <= 2 * NF; ++d) cause = bytemin7(cause, c32[((z + d) * kTileJ + y) * 16 + w]);
      if (cause == 0x7F7F7F7Fu) continue;  // no hole within reach of these 4 nodes
      const int j = j0 + y, k = k0 + z;
      if (j >= G.nj || k >= G.nk) continue;
      const uint8_t* ctr = a8 + ((z + NF) * EJ + (y + NF)) * 4 * EIW + NF + 4 * w;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + 4 * w + q;
        const uint32_t cq = (cause >> (8 * q)) & 0xFFu;
        if (i >= G.ni || cq == 0x7F || ctr[q] != 0x7F) continue;  // out of range, none in reach, or a hole
        // buffer causes are grid ids < 63, so they win over an outer-boundary cause
        fl[(long long)i + (long long)G.ni * ((long long)j + (long long)G.nj * k)] = (uint8_t)(kFringe | (cq << 2));
      }
    }
    __syncthreads();
  }
}

hipError_t launch_fringe(ov_ctx* ctx, int nf, uint8_t* flags, hipStream_t s, int slot, int gen) {
  return launch_fringe_in(ctx, nf, flags, s, ctx_scratch(ctx, slot, gen));
}

hipError_t launch_fringe_in(ov_ctx* ctx, int nf, uint8_t* flags, hipStream_t s, const FrontScratch& fs) {
  const int ng = (int)ctx->grids.size();
  const int4* nl = fs.near_list;
  const int32_t* nc = fs.near_count;
  const unsigned int* st = fs.stamp;
  int32_t* clc = fs.chunk_list_count;
  // persistent blocks over the near list (its length is on the device)
  long long g = std::max(1LL, std::min<long long>(ctx->total_tiles,
                                                    (long long)ctx->num_cus * (ctx->persist > 0 ? ctx->persist : 4)));
#define OV_FRINGE_ARGS                                                                                            \
  ctx->d_grids, ng, flags, nl, nc, st, ctx->d_chunk_static, fs.chunk_stamp, fs.chunk_list, clc, \
      ctx->n_static_chunks
  switch (nf) {
    case 0:
      hipLaunchKernelGGL(k_fringe_tiles<0>, dim3((unsigned)g), dim3(256), 0, s, OV_FRINGE_ARGS);
      break;
    case 1:
      hipLaunchKernelGGL(k_fringe_tiles<1>, dim3((unsigned)g), dim3(256), 0, s, OV_FRINGE_ARGS);
      break;
    case 2:
      hipLaunchKernelGGL(k_fringe_tiles<2>, dim3((unsigned)g), dim3(256), 0, s, OV_FRINGE_ARGS);
      break;
    default:
      hipLaunchKernelGGL(k_fringe_tiles<3>, dim3((unsigned)g), dim3(256), 0, s, OV_FRINGE_ARGS);
      break;
  }
#undef OV_FRINGE_ARGS
  return hipGetLastError();
}

// ================================================================ compaction
// Ordered stream compaction of query nodes over 4096-node chunks (in the
// global node numbering), in three passes. (1) Count each
// listed chunk (the static list of chunks with outer-boundary nodes, then
// this step's list of chunks touching near tiles; no other chunk can hold a
// query node): the count is stored with this step's stamp and added to its
// superchunk of 64 chunks. (2) One block scans the superchunk counts (and
// zeroes them). (3)
// Each listed chunk with queries takes its superchunk's offset plus the
// stamped counts of the lower chunks of its superchunk (one 64-lane load
// and a wavefront sum) and writes its query nodes in node order. Inside a
// chunk a thread owns 16 consecutive flag bytes; the wave prefix of the
// per-thread counts is a shuffle scan and the wave totals are scanned in LDS.
__device__ __forceinline__ int count_fringe16(const uint8_t* p, long long n0, long long total, uint32_t& mask) {
  uint8_t v[16];
  if (n0 + 16 <= total) {
    uint4 q = *reinterpret_cast<const uint4*>(p + n0);
    const uint8_t* b = reinterpret_cast<const uint8_t*>(&q);
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = b[e];
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = (n0 + e < total) ? p[n0 + e] : (uint8_t)0;
  }
  mask = 0;
#pragma unroll
  for (int e = 0; e < 16; ++e) mask |= ((v[e] & 3) == kFringe ? 1u : 0u) << e;
  return __popc(mask);
}

// Exclusive scan of the superchunk counts by one block of up to 1024
// threads (each a contiguous run of superchunks); offsets gets nsuper + 1
// entries, the last the total, which is also the step's query count. The
// counts are zeroed for the next step.
__device__ __forceinline__ void super_scan(int32_t* __restrict__ super_counts, long long nsuper,
                                           long long* __restrict__ offsets, long long* __restrict__ d_count,
                                           long long capacity, int32_t* __restrict__ status) {
  __shared__ long long wtot[1024 / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long per = (nsuper + blockDim.x - 1) / blockDim.x;
  const long long b0 = min(nsuper, (long long)threadIdx.x * per), b1 = min(nsuper, b0 + per);
  auto count_at = [&](long long e) { return (long long)super_counts[e]; };
  long long sum = 0;
  for (long long i = b0; i < b1; ++i)
    for (int q = 0; q < kSuperSlots; ++q) sum += count_at(i * kSuperSlots + q);
  long long inc = sum;
  for (int o = 1; o < 64; o <<= 1) {
    long long t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wtot[wave] = inc;
  __syncthreads();
  long long run = inc - sum;
  for (int w = 0; w < wave; ++w) run += wtot[w];
  for (long long i = b0; i < b1; ++i) {
    offsets[i] = run;
    for (int q = 0; q < kSuperSlots; ++q) {
      run += count_at(i * kSuperSlots + q);
      super_counts[i * kSuperSlots + q] = 0;  // ready for the next step's count
    }
  }
  if (threadIdx.x == blockDim.x - 1) {
    offsets[nsuper] = run;
    *d_count = run;
    if (run > capacity) atomicOr(status, OV_DEV_CAPACITY);
  }
}

// Pass (1): the counts.
__global__ void __launch_bounds__(kCompactThreads) k_compact_count(const uint8_t* __restrict__ flags, long long total,
                                                                   unsigned long long* __restrict__ counts,
                                                                   int32_t* __restrict__ super_counts,
                                                                   const int32_t* __restrict__ chunk_list,
                                                                   const int32_t* __restrict__ chunk_list_count,
                                                                   long long n_static,
                                                                   const unsigned int* __restrict__ d_stamp) {
  __shared__ int red[kCompactThreads / 64];
  // the list length, the stamp and this block's first entry in one round
  // trip (the list has room for every chunk; the grid has no more blocks)
  const long long nl = n_static + *chunk_list_count;
  const unsigned int stamp = *d_stamp;
  const int32_t first = chunk_list[blockIdx.x];
  for (long long e = blockIdx.x; e < nl; e += gridDim.x) {
    const long long ch = e == (long long)blockIdx.x ? first : chunk_list[e];
    uint32_t mask;
    int cnt = count_fringe16(flags, ch * kCompactChunk + threadIdx.x * 16, total, mask);
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_down(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      int sum = 0;
      for (int w = 0; w < kCompactThreads / 64; ++w) sum += red[w];
      counts[ch] = ((unsigned long long)stamp << 32) | (unsigned int)sum;
      if (sum) atomicAdd(&super_counts[(ch / kSuperChunk) * kSuperSlots + ch % kSuperSlots], sum);
    }
    __syncthreads();
  }
}

// Pass (2): the scan, one block.
__global__ void __launch_bounds__(1024) k_compact_scan(int32_t* __restrict__ super_counts, long long nsuper,
                                                      long long* __restrict__ offsets, long long* __restrict__ d_count,
                                                      long long capacity, int32_t* __restrict__ status) {
  super_scan(super_counts, nsuper, offsets, d_count, capacity, status);
}

// The superchunk offsets computed by one block into LDS: exclusive prefix
// sums of the superchunk counts (each thread a contiguous run of
// superchunks), soff[nsuper] = the total. The counts are left as they are.
__device__ __forceinline__ void block_super_prefix(const int32_t* __restrict__ super_counts, long long nsuper,
                                                   long long* soff) {
  __shared__ long long wt[kCompactThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long per = (nsuper + blockDim.x - 1) / blockDim.x;
  const long long b0 = min(nsuper, (long long)threadIdx.x * per), b1 = min(nsuper, b0 + per);
  gmem<int32_t>* sc = gp(super_counts);
  long long sum = 0;
  for (long long i = b0; i < b1; ++i)
    for (int q = 0; q < kSuperSlots; ++q) sum += sc[i * kSuperSlots + q];
  long long inc = sum;
  for (int o = 1; o < 64; o <<= 1) {
    long long t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wt[wave] = inc;
  __syncthreads();
  long long run = inc - sum;
  for (int w = 0; w < wave; ++w) run += wt[w];
  for (long long i = b0; i < b1; ++i) {
    soff[i] = run;
    for (int q = 0; q < kSuperSlots; ++q) run += sc[i * kSuperSlots + q];
  }
  if (threadIdx.x == blockDim.x - 1) soff[nsuper] = run;
}

// Pass (3). FUSED (the step executors): each block first forms the
// superchunk offsets itself (block_super_prefix, in LDS), block 0 stores the
// query count, and no scan kernel runs; the counts are zeroed by the next
// hole cut of the same scratch slot. Otherwise the offsets come from the
// scan kernel.
template <bool FUSED>
__global__ void __launch_bounds__(kCompactThreads) k_compact_write(const GridDev* __restrict__ grids, int ngrids,
                                                                   const uint8_t* __restrict__ flags, long long total,
                                                                   const unsigned long long* __restrict__ counts,
                                                                   long long nchunks,
                                                                   const long long* __restrict__ super_offsets,
                                                                   const int32_t* __restrict__ super_counts,
                                                                   long long nsuper, long long* __restrict__ d_count,
                                                                   int32_t* __restrict__ status,
                                                                   const int32_t* __restrict__ chunk_list,
                                                                   const int32_t* __restrict__ chunk_list_count,
                                                                   long long n_static,
                                                                   const unsigned int* __restrict__ d_stamp,
                                                                   int32_t* __restrict__ q_grid,
                                                                   int32_t* __restrict__ q_node, long long capacity) {
  __shared__ int wsum[kCompactThreads / 64];
  __shared__ long long off[kMaxGrids + 1];
  __shared__ uint16_t qofs[kCompactChunk];  // the chunk's fringe nodes (offsets in the chunk), in order
  extern __shared__ long long soff[];  // FUSED: nsuper + 1 superchunk offsets
  // read up front, beside the superchunk counts: the list length, the stamp
  // and this block's first entry (the list has room for every chunk; the
  // grid has no more blocks)
  const long long nl = n_static + *chunk_list_count;
  const unsigned int stamp = *d_stamp;
  const int32_t first = chunk_list[blockIdx.x];
  for (int g = threadIdx.x; g < ngrids; g += blockDim.x) off[g] = grids[g].node_off;
  if (threadIdx.x == 0) off[ngrids] = total;
  // (a block without a listed chunk skips the prefix; block 0 stores the count)
  if (FUSED && ((long long)blockIdx.x < nl || blockIdx.x == 0)) {
    block_super_prefix(super_counts, nsuper, soff);
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *d_count = soff[nsuper];
      if (soff[nsuper] > capacity) atomicOr(status, OV_DEV_CAPACITY);
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (long long e = blockIdx.x; e < nl; e += gridDim.x) {
    const long long ch = e == (long long)blockIdx.x ? first : chunk_list[e];
    // the chunk's flags, read with its counts (before the test for an empty
    // chunk, so that both loads are in flight together)
    const long long n0 = ch * kCompactChunk + threadIdx.x * 16;
    uint32_t mask;
    const int cnt = count_fringe16(flags, n0, total, mask);
    // this step's counts of the chunks of ch's superchunk below ch (every
    // wavefront forms the same sum)
    const long long c = ch - ch % kSuperChunk + lane;
    const unsigned long long v = (c < ch && c < nchunks) ? counts[c] : 0ull;
    long long below = (unsigned int)(v >> 32) == stamp ? (long long)(unsigned int)v : 0;
    for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o, 64);
    const long long base = (FUSED ? soff[ch / kSuperChunk] : super_offsets[ch / kSuperChunk]) + below;
    const unsigned long long own = counts[ch];
    if ((unsigned int)own == 0u || base >= capacity) continue;  // nothing to write (same in every thread)
    // inclusive wave scan
    int inc = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      int t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < kCompactThreads / 64; ++w) {
      if (w < wave) before += wsum[w];
      tot += wsum[w];
    }
    // the nodes go to LDS in order, then out with consecutive threads on
    // consecutive queries (coalesced stores)
    int p = before + (inc - cnt);
    while (mask) {
      const int q = __ffs(mask) - 1;
      mask &= mask - 1;
      qofs[p++] = (uint16_t)(threadIdx.x * 16 + q);
    }
    __syncthreads();
    const int lim = (int)min((long long)tot, capacity - base);
    const long long c0 = ch * kCompactChunk;
    for (int x = threadIdx.x; x < lim; x += kCompactThreads) {
      const long long n = c0 + qofs[x];
      const int A = grid_of_node(off, ngrids, n);
      q_grid[base + x] = A;
      q_node[base + x] = (int32_t)(n - off[A]);
    }
    __syncthreads();
  }
}

hipError_t launch_compact(ov_ctx* ctx, const uint8_t* flags, int32_t* q_grid, int32_t* q_node, long long capacity,
                          long long* d_count, hipStream_t s, int slot, bool fused) {
  return launch_compact_in(ctx, flags, q_grid, q_node, capacity, d_count, s, ctx_scratch(ctx, slot, 0), fused);
}

hipError_t launch_compact_in(ov_ctx* ctx, const uint8_t* flags, int32_t* q_grid, int32_t* q_node,
                             long long capacity, long long* d_count, hipStream_t s, const FrontScratch& fs,
                             bool fused) {
  const long long total = ctx->node_off.back();
  const unsigned int* st = fs.stamp;
  const int32_t* clc = fs.chunk_list_count;
  int32_t* sc = fs.super_counts;
  // persistent blocks over the chunk list (its length is on the device):
  // as many as the chip holds at once (8 of 256 threads per CU), since each
  // block takes its chunks one after another and every chunk is a chain of
  // dependent memory round trips
  const long long grid = std::max(1LL, std::min<long long>(ctx->nchunks, (long long)ctx->num_cus * 8));
  hipLaunchKernelGGL(k_compact_count, dim3((unsigned)grid), dim3(kCompactThreads), 0, s, flags, total,
                     fs.chunk_counts, sc, fs.chunk_list, clc, ctx->n_static_chunks, st);
  fused = fused && ctx->nsuper <= kFusedScanMax;
  if (!fused)
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, sc, ctx->nsuper, fs.super_offsets, d_count,
                       capacity, ctx->d_status);
#define OV_WRITE_ARGS                                                                                                \
  ctx->d_grids, (int)ctx->grids.size(), flags, total, fs.chunk_counts, ctx->nchunks, fs.super_offsets, sc,           \
      ctx->nsuper, d_count, ctx->d_status, fs.chunk_list, clc, ctx->n_static_chunks, st, q_grid, q_node, capacity
  if (fused)
    hipLaunchKernelGGL(k_compact_write<true>, dim3((unsigned)grid), dim3(kCompactThreads),
                       sizeof(long long) * (ctx->nsuper + 1), s, OV_WRITE_ARGS);
  else
    hipLaunchKernelGGL(k_compact_write<false>, dim3((unsigned)grid), dim3(kCompactThreads), 0, s, OV_WRITE_ARGS);
#undef OV_WRITE_ARGS
  return hipGetLastError();
}

// Chunks holding outer-boundary query nodes (fixed per grid): one block per
// chunk marks them; the host turns the marks into the static chunk list.
__global__ void __launch_bounds__(256) k_chunk_outer(const GridDev* __restrict__ grids, int ngrids, long long total,
                                                    long long nchunks, uint8_t* __restrict__ chunk_static) {
  __shared__ long long off[kMaxGrids + 1];
  for (int g = threadIdx.x; g < ngrids; g += blockDim.x) off[g] = grids[g].node_off;
  if (threadIdx.x == 0) off[ngrids] = total;
  __syncthreads();
  for (long long ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    bool any = false;
    for (int e = threadIdx.x; e < kCompactChunk; e += blockDim.x) {
      const long long n = ch * kCompactChunk + e;
      if (n >= total) break;
      const int A = grid_of_node(off, ngrids, n);
      const GeomR G(grids[A]);
      if (!grids[A].has_outer) continue;
      const long long m = n - off[A];
      const long long plane = (long long)G.ni * G.nj;
      const int k = (int)(m / plane);
      const long long r = m - (long long)k * plane;
      const int j = (int)(r / G.ni), i = (int)(r - (long long)j * G.ni);
      any |= G.on_outer(i, j, k);
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) chunk_static[ch] = any ? 1 : 0;
  }
}

int build_static_chunks(ov_ctx* ctx, hipStream_t s) {
  const long long total = ctx->node_off.back();
  const long long nch = ctx->nchunks;
  long long g = std::max(1LL, std::min(nch, 65536LL));
  hipLaunchKernelGGL(k_chunk_outer, dim3((unsigned)g), dim3(256), 0, s, ctx->d_grids, (int)ctx->grids.size(), total,
                     nch, ctx->d_chunk_static);
  std::vector<uint8_t> marks((size_t)nch);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(marks.data(), ctx->d_chunk_static, (size_t)nch, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "static chunk list");
  std::vector<int32_t> list;
  for (long long c = 0; c < nch; ++c)
    if (marks[(size_t)c]) list.push_back((int32_t)c);
  ctx->n_static_chunks = (long long)list.size();
  // every slot's chunk list starts with the static list
  for (int k = 0; k < kSlots && !list.empty(); ++k) {
    e = hipMemcpy(ctx->d_chunk_list + (long long)k * nch, list.data(), sizeof(int32_t) * list.size(),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "static chunk list upload");
  }
  return OV_OK;
}

// ================================================================ transform
// The query's offset from its grid's frame centre in inertial axes,
// x - c_g = R_g X_g. Consumers add c_g in FP64, so in mixed precision the
// FP32 value carries only the small body-scale offset.
template <typename T>
__global__ void k_transform(const GridDev* __restrict__ grids, const double* __restrict__ poses,
                            const int32_t* __restrict__ q_grid, const int32_t* __restrict__ q_node,
                            const long long* __restrict__ d_count, long long capacity, T* __restrict__ qx) {
  long long n = min(*d_count, capacity);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    const int g = q_grid[q];
    T o[3];
    transform_node<T>(grids[g], poses + 12 * g, q_node[q], o);
    qx[q] = o[0];
    qx[capacity + q] = o[1];
    qx[2 * capacity + q] = o[2];
  }
}

hipError_t launch_transform(ov_ctx* ctx, const double* poses, const int32_t* q_grid, const int32_t* q_node,
                            const long long* d_count, long long capacity, void* qx, hipStream_t s) {
  const int block = 256;
  long long grid = grid_size_for(ctx, capacity, block);
  if (ctx->precision == OV_MIXED)
    hipLaunchKernelGGL(k_transform<float>, dim3((unsigned)grid), dim3(block), 0, s, ctx->d_grids, poses, q_grid,
                       q_node, d_count, capacity, (float*)qx);
  else
    hipLaunchKernelGGL(k_transform<double>, dim3((unsigned)grid), dim3(block), 0, s, ctx->d_grids, poses, q_grid,
                       q_node, d_count, capacity, (double*)qx);
  return hipGetLastError();
}

// ================================================================ interpolation
// One query per thread: the donor cell's 8 corner nodes (periodic wrap), the
// trilinear weights w_c = prod_d (c_d ? s_d : 1 - s_d), and the gathered sum
// for each of the 4 fields.
template <typename T>
__global__ void k_interp(const GridDev* __restrict__ grids, const int32_t* __restrict__ donor_grid,
                         const int32_t* __restrict__ donor_cell, const T* __restrict__ s,
                         const long long* __restrict__ d_count, long long capacity, const T* __restrict__ fields,
                         long long total_nodes, int interleaved, T* __restrict__ out) {
  long long n = min(*d_count, capacity);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    int B = donor_grid[q];
    if (B < 0) continue;
    T v[4];
    interp_point<T>(grids[B], donor_cell[q], s[q], s[capacity + q], s[2 * capacity + q], fields, total_nodes,
                    interleaved != 0, v);
#pragma unroll
    for (int f = 0; f < 4; ++f) out[(long long)f * capacity + q] = v[f];
  }
}

hipError_t launch_interp(ov_ctx* ctx, const int32_t* donor_grid, const int32_t* donor_cell, const void* s,
                         const long long* d_count, long long capacity, const void* fields, void* out, hipStream_t st) {
  int block = ctx->interp_block;
  long long grid = grid_size_for(ctx, capacity, block);
  long long total = ctx->node_off.back();
  if (ctx->precision == OV_MIXED)
    hipLaunchKernelGGL(k_interp<float>, dim3((unsigned)grid), dim3(block), 0, st, ctx->d_grids, donor_grid,
                       donor_cell, (const float*)s, d_count, capacity, (const float*)fields, total,
                       ctx->field_layout, (float*)out);
  else
    hipLaunchKernelGGL(k_interp<double>, dim3((unsigned)grid), dim3(block), 0, st, ctx->d_grids, donor_grid,
                       donor_cell, (const double*)s, d_count, capacity, (const double*)fields, total,
                       ctx->field_layout, (double*)out);
  return hipGetLastError();
}

}  // namespace ov

using namespace ov;

// ================================================================ C ABI (step)
static int ready(ov_ctx* ctx) {
  if (!ctx) return OV_EINVAL;
  if (!ctx->finalized) return fail(ctx, OV_ESTATE, "step call before ov_finalize");
  return OV_OK;
}

static int launched(ov_ctx* ctx, hipError_t e, const char* what) {
  return e == hipSuccess ? OV_OK : hip_fail(ctx, e, what);
}

extern "C" {

int overset_holecut(ov_ctx* ctx, const double* poses, uint8_t* flags, void* stream) {
  int rc = ready(ctx);
  if (rc) return rc;
  if (!poses || !flags) return fail(ctx, OV_EINVAL, "overset_holecut: null pointer");
  return launched(ctx, launch_holecut(ctx, poses, flags, (hipStream_t)stream), "overset_holecut");
}

int overset_fringe_compact(ov_ctx* ctx, int32_t nf, uint8_t* flags, int32_t* q_grid, int32_t* q_node,
                           int64_t capacity, int64_t* d_count, void* stream) {
  int rc = ready(ctx);
  if (rc) return rc;
  if (!flags || !d_count || (capacity > 0 && (!q_grid || !q_node)))
    return fail(ctx, OV_EINVAL, "overset_fringe_compact: null pointer");
  if (((uintptr_t)flags & 15) != 0) return fail(ctx, OV_EINVAL, "overset_fringe_compact: flags must be 16-byte aligned");
  if (nf < 0 || nf > kMaxNf) return fail(ctx, OV_EINVAL, "overset_fringe_compact: nf must be in 0..%d", kMaxNf);
  if (capacity < 0) return fail(ctx, OV_EINVAL, "overset_fringe_compact: negative capacity");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_near_from_flags(ctx, flags, s);
  if (e == hipSuccess) e = launch_fringe(ctx, nf, flags, s);
  if (e == hipSuccess) e = launch_compact(ctx, flags, q_grid, q_node, capacity, (long long*)d_count, s);
  return launched(ctx, e, "overset_fringe_compact");
}

int overset_transform(ov_ctx* ctx, const double* poses, const int32_t* q_grid, const int32_t* q_node,
                      const int64_t* d_count, int64_t capacity, void* qx, void* stream) {
  int rc = ready(ctx);
  if (rc) return rc;
  if (capacity < 0) return fail(ctx, OV_EINVAL, "overset_transform: negative capacity");
  if (capacity == 0) return OV_OK;
  if (!poses || !q_grid || !q_node || !d_count || !qx) return fail(ctx, OV_EINVAL, "overset_transform: null pointer");
  return launched(ctx,
                  launch_transform(ctx, poses, q_grid, q_node, (const long long*)d_count, capacity, qx,
                                   (hipStream_t)stream),
                  "overset_transform");
}

int overset_interp(ov_ctx* ctx, const int32_t* donor_grid, const int32_t* donor_cell, const void* s,
                   const int64_t* d_count, int64_t capacity, const void* fields, void* out, void* stream) {
  int rc = ready(ctx);
  if (rc) return rc;
  if (capacity < 0) return fail(ctx, OV_EINVAL, "overset_interp: negative capacity");
  if (capacity == 0) return OV_OK;
  if (!donor_grid || !donor_cell || !s || !d_count || !fields || !out)
    return fail(ctx, OV_EINVAL, "overset_interp: null pointer");
  return launched(ctx,
                  launch_interp(ctx, donor_grid, donor_cell, s, (const long long*)d_count, capacity, fields, out,
                                (hipStream_t)stream),
                  "overset_interp");
}

}  // extern "C"
