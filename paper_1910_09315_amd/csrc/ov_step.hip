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
  int blank[kMaxGrids];
  int kind[kMaxGrids];
  int outer[kMaxGrids];
  int nblank;
};

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
    } else if (G.blank_kind != OV_BLANK_NONE) {
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
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nb = 0;
    for (int g = 0; g < ngrids; ++g)
      if (L.kind[g] != OV_BLANK_NONE) L.blank[nb++] = g;
    L.nblank = nb;
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
  if (kind == OV_BLANK_CYL) {
    double r = prm[0];
    return (x * x + y * y) < r * r && z >= prm[1] && z <= prm[2];
  }
  if (kind == OV_BLANK_SPHERE) return (x * x + y * y + z * z) < prm[0] * prm[0];
  double u = x / prm[0], v = y / prm[1], w = z / prm[2];
  return (u * u + v * v + w * w) < 1.0;
}

// FP64 decision for one node of grid A at world position w: first blanking grid or -1.
__device__ __forceinline__ int holecut_fp64(const HoleLds& L, int A, const double w[3]) {
  for (int b = 0; b < L.nblank; ++b) {
    int B = L.blank[b];
    if (B == A) continue;
    const double* p = L.pose[B];
    double d0 = w[0] - p[9], d1 = w[1] - p[10], d2 = w[2] - p[11];
    if (d0 * d0 + d1 * d1 + d2 * d2 >= L.cull[B]) continue;
    double x = p[0] * d0 + p[3] * d1 + p[6] * d2;
    double y = p[1] * d0 + p[4] * d1 + p[7] * d2;
    double z = p[2] * d0 + p[5] * d1 + p[8] * d2;
    if (blank_inside_fp64(L.kind[B], L.prm[B], x, y, z)) return B;
  }
  return -1;
}

// FP32 guard band: nodes whose FP32 inside measure is within this of the
// surface are decided again in FP64 from the FP64 coordinates.
constexpr float kHoleGuard = 1e-3f;

// Streaming hole cut: each thread loads the coordinates of NPT nodes (strided
// by the block size, so every load instruction is coalesced) before testing
// any of them, which keeps 3 * NPT loads per lane in flight.
template <typename CT>
__device__ __forceinline__ int holecut_node(const HoleLds& L, const GridDev* __restrict__ grids, int A, long long m,
                                            CT X, CT Y, CT Z) {
  const double* pa = L.pose[A];
  if (sizeof(CT) == 8) {
    double w[3];
    w[0] = pa[0] * X + pa[1] * Y + pa[2] * Z + pa[9];
    w[1] = pa[3] * X + pa[4] * Y + pa[5] * Z + pa[10];
    w[2] = pa[6] * X + pa[7] * Y + pa[8] * Z + pa[11];
    return holecut_fp64(L, A, w);
  }
  const float* pf = L.posef[A];
  const float Xf = (float)X, Yf = (float)Y, Zf = (float)Z;
  float w0 = pf[0] * Xf + pf[1] * Yf + pf[2] * Zf + pf[9];
  float w1 = pf[3] * Xf + pf[4] * Yf + pf[5] * Zf + pf[10];
  float w2 = pf[6] * Xf + pf[7] * Yf + pf[8] * Zf + pf[11];
  bool unsure = false;
  int cause = -1;
  for (int b = 0; b < L.nblank; ++b) {
    int B = L.blank[b];
    if (B == A) continue;
    const float* p = L.posef[B];
    float d0 = w0 - p[9], d1 = w1 - p[10], d2 = w2 - p[11];
    if (d0 * d0 + d1 * d1 + d2 * d2 >= L.cullf[B]) continue;
    float x = p[0] * d0 + p[3] * d1 + p[6] * d2;
    float y = p[1] * d0 + p[4] * d1 + p[7] * d2;
    float z = p[2] * d0 + p[5] * d1 + p[8] * d2;
    float f = blank_measure_f32(L.kind[B], L.prmf[B], x, y, z);
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
    double Xd = G.X[m], Yd = G.Y[m], Zd = G.Z[m];
    double w[3];
    w[0] = pa[0] * Xd + pa[1] * Yd + pa[2] * Zd + pa[9];
    w[1] = pa[3] * Xd + pa[4] * Yd + pa[5] * Zd + pa[10];
    w[2] = pa[6] * Xd + pa[7] * Yd + pa[8] * Zd + pa[11];
    cause = holecut_fp64(L, A, w);
  }
  return cause;
}

// Flag byte of a node given its hole cause (-1: none). Holes mark their
// fringe tile in the tile map; nodes of grids with outer layers compute their
// (i, j, k) to mark the outer-boundary query layers (a fixed set per grid).
// Grid geometry kept in registers by loops that store flag bytes (a byte
// store may alias anything, so fields read through a GridDev reference would
// be re-loaded after every store).
struct GeomR {
  int ni, nj, nk, tiles_i, tiles_j;
  int o0, o1, o2, o3, o4, o5;
  long long tile_off;
  __device__ __forceinline__ explicit GeomR(const GridDev& G)
      : ni(G.ni), nj(G.nj), nk(G.nk), tiles_i(G.tiles_i), tiles_j(G.tiles_j), o0(G.outer[0]), o1(G.outer[1]),
        o2(G.outer[2]), o3(G.outer[3]), o4(G.outer[4]), o5(G.outer[5]), tile_off(G.tile_off) {}
  __device__ __forceinline__ bool on_outer(int i, int j, int k) const {
    return i < o0 || i >= ni - o1 || j < o2 || j >= nj - o3 || k < o4 || k >= nk - o5;
  }
};

__device__ __forceinline__ uint8_t node_flag(const GeomR& G, long long m, int cause, uint8_t* tile_hole) {
  long long plane = (long long)G.ni * G.nj;
  int k = (int)(m / plane);
  long long r = m - (long long)k * plane;
  int j = (int)(r / G.ni);
  int i = (int)(r - (long long)j * G.ni);
  if (cause >= 0) {
    tile_hole[G.tile_off + (i >> 6) + (long long)G.tiles_i * ((j >> 3) + (long long)G.tiles_j * (k >> 3))] = 1;
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
                                                 long long total_chunks, uint8_t* __restrict__ tile_hole,
                                                 unsigned long long* __restrict__ stats) {
  typedef typename Vec16<CT>::type V;
  constexpr int W = Vec16<CT>::W;
  __shared__ HoleLds L;
  __shared__ long long coff[kMaxGrids + 1];  // first chunk of each grid
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
      atomicAdd(&stats[OV_STAT_HOLECUT_NODES_READ], (unsigned long long)L.off[ngrids]);
      atomicAdd(&stats[OV_STAT_HOLECUT_CALLS], 1ULL);
    }
  }
  __syncthreads();
  for (long long ch = blockIdx.x; ch < total_chunks; ch += gridDim.x) {
    const int A = grid_of_node(coff, ngrids, ch);
    const long long nn = L.off[A + 1] - L.off[A];
    const long long m0 = (ch - coff[A]) * span + (long long)threadIdx.x * W;
    const CT* Xa = (const CT*)L.X[A];
    const CT* Ya = (const CT*)L.Y[A];
    const CT* Za = (const CT*)L.Z[A];
    uint8_t* fa = flags + L.off[A];
    const GeomR GR(grids[A]);
    const bool outerA = L.outer[A] != 0;
    CT X[R][W], Y[R][W], Z[R][W];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long m = m0 + (long long)r * blockDim.x * W;
      if (m + W <= nn) {
        V x = __builtin_nontemporal_load(reinterpret_cast<const V*>(Xa + m));
        V y = __builtin_nontemporal_load(reinterpret_cast<const V*>(Ya + m));
        V z = __builtin_nontemporal_load(reinterpret_cast<const V*>(Za + m));
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
        int cause = holecut_node<CT>(L, grids, A, m + w, X[r][w], Y[r][w], Z[r][w]);
        fa[m + w] = (cause < 0 && !outerA) ? (uint8_t)OV_STATE_FIELD : node_flag(GR, m + w, cause, tile_hole);
      }
    }
  }
}

static_assert(kTileI == 64 && kTileJ == 8 && kTileK == 8 && 256 * 16 == kTileI * kTileJ * kTileK,
              "a 256-thread block covers a tile with 16 bytes per thread");

// Hole cut over node tiles (kTileI x kTileJ x kTileK, one block per tile)
// with culling: a tile whose bounding sphere, placed at its grid's pose,
// cannot reach the bounding sphere of any other grid's blank region holds no
// hole, so its coordinates are not read; its flags are still written (field,
// or fringe on outer-boundary layers). Tiles that may be cut test every node
// exactly as the streaming kernel does. The kernel also records, for every
// tile, whether it holds a hole (the fringe pass reads that map).
template <typename CT>
__global__ void __launch_bounds__(256) k_holecut_tiles(const GridDev* __restrict__ grids, int ngrids,
                                                      const double* __restrict__ poses, uint8_t* __restrict__ flags,
                                                      const double4* __restrict__ spheres, long long total_tiles,
                                                      uint8_t* __restrict__ tile_hole,
                                                      unsigned long long* __restrict__ stats) {
  __shared__ HoleLds L;
  __shared__ long long toff[kMaxGrids + 1];
  holecut_stage<CT>(L, grids, ngrids, poses);
  for (int g = threadIdx.x; g < ngrids; g += blockDim.x) toff[g] = grids[g].tile_off;
  if (threadIdx.x == 0) toff[ngrids] = total_tiles;
  __syncthreads();
  for (long long tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    const int A = grid_of_node(toff, ngrids, tile);
    const GeomR G(grids[A]);
    const int t = (int)(tile - toff[A]);
    const int i0 = (t % G.tiles_i) * kTileI;
    const int j0 = ((t / G.tiles_i) % G.tiles_j) * kTileJ;
    const int k0 = (t / (G.tiles_i * G.tiles_j)) * kTileK;
    // may any blank region reach this tile? (the same answer in every thread)
    const double4 sp = spheres[tile];
    const double* pa = L.pose[A];
    const double wc0 = pa[0] * sp.x + pa[1] * sp.y + pa[2] * sp.z + pa[9];
    const double wc1 = pa[3] * sp.x + pa[4] * sp.y + pa[5] * sp.z + pa[10];
    const double wc2 = pa[6] * sp.x + pa[7] * sp.y + pa[8] * sp.z + pa[11];
    bool cand = false;
    for (int b = 0; b < L.nblank; ++b) {
      const int B = L.blank[b];
      if (B == A) continue;
      const double* p = L.pose[B];
      const double d0 = wc0 - p[9], d1 = wc1 - p[10], d2 = wc2 - p[11];
      const double rr = (sqrt(L.cull[B]) + sp.w) * (1.0 + 1e-9) + 1e-12;
      cand |= d0 * d0 + d1 * d1 + d2 * d2 <= rr * rr;
    }
    if (tile == blockIdx.x && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&stats[OV_STAT_HOLECUT_CALLS], 1ULL);
    if (cand && threadIdx.x == 0) {
      unsigned long long n = (unsigned long long)min(kTileI, G.ni - i0) * min(kTileJ, G.nj - j0) * min(kTileK, G.nk - k0);
      atomicAdd(&stats[OV_STAT_HOLECUT_NODES_READ], n);
    }
    uint8_t* fa = flags + L.off[A];
    const CT* Xa = (const CT*)L.X[A];
    const CT* Ya = (const CT*)L.Y[A];
    const CT* Za = (const CT*)L.Z[A];
    const bool outer = L.outer[A] != 0;
    bool hole = false;
    if (!cand) {
      // no hole possible: each thread writes 16 flag bytes of one tile row
      const int row = threadIdx.x >> 2, part = threadIdx.x & 3;
      const int i = i0 + part * 16, j = j0 + (row & 7), k = k0 + (row >> 3);
      if (threadIdx.x < 256 && i < G.ni && j < G.nj && k < G.nk) {
        const long long m = (long long)i + (long long)G.ni * ((long long)j + (long long)G.nj * k);
        uint8_t* dst = fa + m;
        const int n = min(16, G.ni - i);
        const bool row_outer = outer && (j < G.o2 || j >= G.nj - G.o3 || k < G.o4 || k >= G.nk - G.o5);
        if (!outer || (!row_outer && i >= G.o0 && i + 16 <= G.ni - G.o1)) {
          if (n == 16 && (((uintptr_t)dst) & 15) == 0) {
            *reinterpret_cast<uint4*>(dst) = make_uint4(0u, 0u, 0u, 0u);
          } else {
            for (int q = 0; q < n; ++q) dst[q] = (uint8_t)OV_STATE_FIELD;
          }
        } else {
          for (int q = 0; q < n; ++q)
            dst[q] = (row_outer || i + q < G.o0 || i + q >= G.ni - G.o1) ? (uint8_t)(kFringe | (OV_CAUSE_BOUNDARY << 2))
                                                                           : (uint8_t)OV_STATE_FIELD;
        }
      }
    } else {
    // 4 nodes per batch: their coordinates are loaded before any flag store
    for (int e0 = threadIdx.x; e0 < kTileI * kTileJ * kTileK; e0 += 4 * blockDim.x) {
      long long m[4];
      bool ok[4], onb[4];
      CT X[4], Y[4], Z[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = e0 + r * blockDim.x;
        const int i = i0 + (e & 63), j = j0 + ((e >> 6) & 7), k = k0 + (e >> 9);
        ok[r] = e < kTileI * kTileJ * kTileK && i < G.ni && j < G.nj && k < G.nk;
        m[r] = (long long)i + (long long)G.ni * ((long long)j + (long long)G.nj * k);
        onb[r] = outer && G.on_outer(i, j, k);
        if (cand && ok[r]) {
          X[r] = Xa[m[r]];
          Y[r] = Ya[m[r]];
          Z[r] = Za[m[r]];
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (!ok[r]) continue;
        const int cause = cand ? holecut_node<CT>(L, grids, A, m[r], X[r], Y[r], Z[r]) : -1;
        uint8_t f = (uint8_t)OV_STATE_FIELD;
        if (cause >= 0) {
          f = (uint8_t)(kHole | (cause << 2));
          hole = true;
        } else if (onb[r]) {
          f = (uint8_t)(kFringe | (OV_CAUSE_BOUNDARY << 2));
        }
        fa[m[r]] = f;
      }
    }
    }
    hole = __syncthreads_or(hole);
    if (threadIdx.x == 0) tile_hole[tile] = hole ? 1 : 0;
  }
}

template <typename CT>
static void launch_holecut_t(ov_ctx* ctx, const double* poses, uint8_t* flags, hipStream_t s) {
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
                       chunks, ctx->d_tile_hole, ctx->d_stats);
  else if (R == 2)
    hipLaunchKernelGGL((k_holecut<CT, 2>), dim3((unsigned)grid), dim3(block), 0, s, ctx->d_grids, ng, poses, flags,
                       chunks, ctx->d_tile_hole, ctx->d_stats);
  else
    hipLaunchKernelGGL((k_holecut<CT, 1>), dim3((unsigned)grid), dim3(block), 0, s, ctx->d_grids, ng, poses, flags,
                       chunks, ctx->d_tile_hole, ctx->d_stats);
}

hipError_t launch_holecut(ov_ctx* ctx, const double* poses, uint8_t* flags, hipStream_t s) {
  if (ctx->cull) {
    int per_cu = ctx->persist > 0 ? ctx->persist : 8;
    long long grid = std::max(1LL, std::min(ctx->total_tiles, (long long)ctx->num_cus * per_cu));
    int ng = (int)ctx->grids.size();
    if (ctx->precision == OV_MIXED)
      hipLaunchKernelGGL(k_holecut_tiles<float>, dim3((unsigned)grid), dim3(256), 0, s, ctx->d_grids, ng, poses,
                         flags, (const double4*)ctx->d_tile_sphere, ctx->total_tiles, ctx->d_tile_hole,
                         ctx->d_stats);
    else
      hipLaunchKernelGGL(k_holecut_tiles<double>, dim3((unsigned)grid), dim3(256), 0, s, ctx->d_grids, ng, poses,
                         flags, (const double4*)ctx->d_tile_sphere, ctx->total_tiles, ctx->d_tile_hole,
                         ctx->d_stats);
    return hipGetLastError();
  }
  if (ctx->precision == OV_MIXED) launch_holecut_t<float>(ctx, poses, flags, s);
  else launch_holecut_t<double>(ctx, poses, flags, s);
  return hipGetLastError();
}

// ================================================================ fringe marking
// The hole cut already wrote holes, the outer-boundary layers and, per 3D
// tile of kTileI x kTileJ x kTileK nodes, whether the tile holds a hole.
// Only tiles with a hole in themselves or a neighbour tile (nf < tile size,
// so the buffer reaches no further) can gain buffer nodes: a block checks
// the 27 map entries of its tile and leaves at once otherwise; near a hole it
// stages the tile plus an nf halo in LDS as "cause if hole, 255 otherwise"
// and takes the lowest cause within Chebyshev distance nf by a separable min
// filter (i, then j, then k).
// Holes are never rewritten, so updating flags in place is race-free: a
// neighbour tile only reads whether a node is a hole.
static_assert(kTileI == 64 && kTileJ == 8 && kTileK == 8, "tile indexing below uses shifts");

__device__ __forceinline__ int wrap_or_out(int v, int n, bool periodic) {
  if (v >= 0 && v < n) return v;
  if (!periodic) return -1;
  v %= n;
  return v < 0 ? v + n : v;
}

__device__ __forceinline__ int tile_grid(const GridDev* __restrict__ grids, int ngrids, long long tile) {
  int lo = 0, hi = ngrids - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (grids[mid].tile_off <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ void tile_coords(const GridDev& G, long long tile, int& ti, int& tj, int& tk) {
  long long t = tile - G.tile_off;
  ti = (int)(t % G.tiles_i);
  tj = (int)((t / G.tiles_i) % G.tiles_j);
  tk = (int)(t / ((long long)G.tiles_i * G.tiles_j));
}

template <int NF>
__global__ void __launch_bounds__(256) k_fringe_tiles(const GridDev* __restrict__ grids, int ngrids,
                                                     uint8_t* __restrict__ flags, const uint8_t* __restrict__ tile_hole,
                                                     long long total_tiles) {
  constexpr int EI = kTileI + 2 * NF, EJ = kTileJ + 2 * NF, EK = kTileK + 2 * NF;
  constexpr int NROW = EJ * EK * 16, NHALO = EJ * EK * 2 * NF;
  __shared__ uint8_t a[EK][EJ][EI];
  __shared__ uint8_t b[EK][EJ][kTileI];
  __shared__ uint8_t c[EK][kTileJ][kTileI];
  for (long long tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    const GridDev& GD = grids[tile_grid(grids, ngrids, tile)];
    int ti, tj, tk;
    tile_coords(GD, tile, ti, tj, tk);
    struct {
      int ni, nj, nk, per, tiles_i, tiles_j, tiles_k;
    } const G = {GD.ni, GD.nj, GD.nk, GD.per, GD.tiles_i, GD.tiles_j, GD.tiles_k};
    const long long toff = GD.tile_off;
    // a hole in this tile or a neighbour tile? (nf < tile size: nothing further matters)
    bool near = false;
    if (threadIdx.x < 27) {
      int x = wrap_or_out(ti + (int)threadIdx.x % 3 - 1, G.tiles_i, G.per & 1);
      int y = wrap_or_out(tj + ((int)threadIdx.x / 3) % 3 - 1, G.tiles_j, G.per & 2);
      int z = wrap_or_out(tk + (int)threadIdx.x / 9 - 1, G.tiles_k, G.per & 4);
      if (x >= 0 && y >= 0 && z >= 0) near = tile_hole[toff + x + (long long)G.tiles_i * (y + (long long)G.tiles_j * z)];
    }
    if (!__syncthreads_or(near)) continue;
    const int i0 = ti * kTileI, j0 = tj * kTileJ, k0 = tk * kTileK;
    uint8_t* fl = flags + GD.node_off;
    // stage hole causes with halo: 16 threads per row load the 64 interior
    // bytes as words where the row is aligned and in range, the halo bytewise;
    // fixed trip counts so that all loads are issued before the LDS stores
#pragma unroll
    for (int it = 0; it < (NROW + 255) / 256; ++it) {
      const int e = threadIdx.x + it * 256;
      if (e >= NROW) break;
      const int row = e >> 4, part = e & 15;
      const int y = row % EJ, z = row / EJ;
      const int j = wrap_or_out(j0 - NF + y, G.nj, G.per & 2);
      const int k = wrap_or_out(k0 - NF + z, G.nk, G.per & 4);
      uint8_t v[4] = {255, 255, 255, 255};
      if (j >= 0 && k >= 0) {
        const uint8_t* rowp = fl + (long long)G.ni * ((long long)j + (long long)G.nj * k);
        const int i = i0 + part * 4;
        if (i + 4 <= G.ni && (((uintptr_t)(rowp + i)) & 3) == 0) {
          uint32_t w4 = *reinterpret_cast<const uint32_t*>(rowp + i);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            uint8_t f = (uint8_t)(w4 >> (8 * q));
            v[q] = ((f & 3) == kHole) ? (uint8_t)(f >> 2) : (uint8_t)255;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            int ii = wrap_or_out(i + q, G.ni, G.per & 1);
            if (ii >= 0) {
              uint8_t f = rowp[ii];
              if ((f & 3) == kHole) v[q] = f >> 2;
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) a[z][y][NF + part * 4 + q] = v[q];
    }
#pragma unroll
    for (int it = 0; it < (NHALO + 255) / 256; ++it) {
      const int e = threadIdx.x + it * 256;
      if (e >= NHALO) break;
      const int h = e % (2 * NF), row = e / (2 * NF);
      const int y = row % EJ, z = row / EJ;
      const int x = h < NF ? h : kTileI + h;  // NF halo bytes on each side
      const int i = wrap_or_out(i0 - NF + x, G.ni, G.per & 1);
      const int j = wrap_or_out(j0 - NF + y, G.nj, G.per & 2);
      const int k = wrap_or_out(k0 - NF + z, G.nk, G.per & 4);
      uint8_t v = 255;
      if (i >= 0 && j >= 0 && k >= 0) {
        uint8_t f = fl[(long long)i + (long long)G.ni * ((long long)j + (long long)G.nj * k)];
        if ((f & 3) == kHole) v = f >> 2;
      }
      a[z][y][x] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kTileI * EJ * EK; e += blockDim.x) {
      int x = e & 63, y = (e >> 6) % EJ, z = (e >> 6) / EJ;
      uint8_t m = 255;
#pragma unroll
      for (int d = 0; d <= 2 * NF; ++d) m = min(m, a[z][y][x + d]);
      b[z][y][x] = m;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kTileI * kTileJ * EK; e += blockDim.x) {
      int x = e & 63, y = (e >> 6) & 7, z = e >> 9;
      uint8_t m = 255;
#pragma unroll
      for (int d = 0; d <= 2 * NF; ++d) m = min(m, b[z][y + d][x]);
      c[z][y][x] = m;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kTileI * kTileJ * kTileK; e += blockDim.x) {
      int x = e & 63, y = (e >> 6) & 7, z = e >> 9;
      int i = i0 + x, j = j0 + y, k = k0 + z;
      if (i >= G.ni || j >= G.nj || k >= G.nk) continue;
      if (a[z + NF][y + NF][x + NF] != 255) continue;  // a hole (staged above)
      uint8_t cause = 255;
#pragma unroll
      for (int d = 0; d <= 2 * NF; ++d) cause = min(cause, c[z + d][y][x]);
      if (cause == 255) continue;
      // buffer causes are grid ids < 63, so they win over an outer-boundary cause
      fl[(long long)i + (long long)G.ni * ((long long)j + (long long)G.nj * k)] = (uint8_t)(kFringe | (cause << 2));
    }
    __syncthreads();
  }
}

hipError_t launch_fringe(ov_ctx* ctx, int nf, uint8_t* flags, hipStream_t s) {
  if (nf == 0) return hipSuccess;  // outer layers were marked by the hole cut
  const int ng = (int)ctx->grids.size();
  long long g = std::max(1LL, std::min<long long>(ctx->total_tiles, (long long)ctx->num_cus * 8));
  switch (nf) {
    case 1:
      hipLaunchKernelGGL(k_fringe_tiles<1>, dim3((unsigned)g), dim3(256), 0, s, ctx->d_grids, ng, flags,
                         ctx->d_tile_hole, ctx->total_tiles);
      break;
    case 2:
      hipLaunchKernelGGL(k_fringe_tiles<2>, dim3((unsigned)g), dim3(256), 0, s, ctx->d_grids, ng, flags,
                         ctx->d_tile_hole, ctx->total_tiles);
      break;
    default:
      hipLaunchKernelGGL(k_fringe_tiles<3>, dim3((unsigned)g), dim3(256), 0, s, ctx->d_grids, ng, flags,
                         ctx->d_tile_hole, ctx->total_tiles);
      break;
  }
  return hipGetLastError();
}

// ================================================================ compaction
// Ordered stream compaction of fringe nodes in three passes over 4096-node
// chunks: count per chunk, exclusive scan of the counts (one block), then
// each chunk writes its fringe nodes at its offset in node order. Inside a
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

__global__ void __launch_bounds__(kCompactThreads) k_compact_count(const uint8_t* __restrict__ flags, long long total,
                                                                   int32_t* __restrict__ counts, long long nchunks,
                                                                   uint8_t* __restrict__ tile_hole, long long ntiles) {
  __shared__ int red[kCompactThreads / 64];
  // the fringe pass has consumed the tile map: clear it for the next hole cut
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += (long long)gridDim.x * blockDim.x)
    tile_hole[t] = 0;
  for (long long ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    uint32_t mask;
    int cnt = count_fringe16(flags, ch * kCompactChunk + threadIdx.x * 16, total, mask);
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_down(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      int sum = 0;
      for (int w = 0; w < kCompactThreads / 64; ++w) sum += red[w];
      counts[ch] = sum;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024) k_compact_scan(const int32_t* __restrict__ counts, long long n,
                                                      long long* __restrict__ offsets, long long* __restrict__ d_count,
                                                      long long capacity, int32_t* __restrict__ status) {
  __shared__ long long part[1024];
  long long per = (n + blockDim.x - 1) / blockDim.x;
  long long b0 = threadIdx.x * per, b1 = min(n, b0 + per);
  long long sum = 0;
  for (long long i = b0; i < b1; ++i) sum += counts[i];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {
    long long v = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  long long run = part[threadIdx.x] - sum;
  for (long long i = b0; i < b1; ++i) {
    offsets[i] = run;
    run += counts[i];
  }
  if (threadIdx.x == blockDim.x - 1) {
    long long total = part[threadIdx.x];
    *d_count = total;
    if (total > capacity) atomicOr(status, OV_DEV_CAPACITY);
  }
}

__global__ void __launch_bounds__(kCompactThreads) k_compact_write(const GridDev* __restrict__ grids, int ngrids,
                                                                   const uint8_t* __restrict__ flags, long long total,
                                                                   const long long* __restrict__ offsets,
                                                                   long long nchunks, int32_t* __restrict__ q_grid,
                                                                   int32_t* __restrict__ q_node, long long capacity) {
  __shared__ int wsum[kCompactThreads / 64];
  __shared__ long long off[kMaxGrids + 1];
  for (int g = threadIdx.x; g < ngrids; g += blockDim.x) off[g] = grids[g].node_off;
  if (threadIdx.x == 0) off[ngrids] = total;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (long long ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    long long n0 = ch * kCompactChunk + threadIdx.x * 16;
    uint32_t mask;
    int cnt = count_fringe16(flags, n0, total, mask);
    // inclusive wave scan
    int inc = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      int v = __shfl_up(inc, o, 64);
      if (lane >= o) inc += v;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    long long pos = offsets[ch] + before + (inc - cnt);
    while (mask) {
      int e = __ffs(mask) - 1;
      mask &= mask - 1;
      if (pos < capacity) {
        long long n = n0 + e;
        int A = grid_of_node(off, ngrids, n);
        q_grid[pos] = A;
        q_node[pos] = (int32_t)(n - off[A]);
      }
      ++pos;
    }
    __syncthreads();
  }
}

hipError_t launch_compact(ov_ctx* ctx, const uint8_t* flags, int32_t* q_grid, int32_t* q_node, long long capacity,
                          long long* d_count, hipStream_t s) {
  long long total = ctx->node_off.back();
  long long nch = ctx->nchunks;
  long long grid = nch;
  if (ctx->persist > 0) grid = std::min<long long>(grid, (long long)ctx->num_cus * ctx->persist);
  hipLaunchKernelGGL(k_compact_count, dim3((unsigned)grid), dim3(kCompactThreads), 0, s, flags, total,
                     ctx->d_chunk_counts, nch, ctx->d_tile_hole, ctx->total_tiles);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, ctx->d_chunk_counts, nch, ctx->d_chunk_offsets,
                     d_count, capacity, ctx->d_status);
  hipLaunchKernelGGL(k_compact_write, dim3((unsigned)grid), dim3(kCompactThreads), 0, s, ctx->d_grids,
                     (int)ctx->grids.size(), flags, total, ctx->d_chunk_offsets, nch, q_grid, q_node, capacity);
  return hipGetLastError();
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
    int g = q_grid[q];
    long long m = q_node[q];
    const GridDev& G = grids[g];
    const double* p = poses + 12 * g;
    if (sizeof(T) == 8) {
      double X = G.X[m], Y = G.Y[m], Z = G.Z[m];
      qx[q] = (T)(p[0] * X + p[1] * Y + p[2] * Z);
      qx[capacity + q] = (T)(p[3] * X + p[4] * Y + p[5] * Z);
      qx[2 * capacity + q] = (T)(p[6] * X + p[7] * Y + p[8] * Z);
    } else {
      float X = G.Xf[m], Y = G.Yf[m], Z = G.Zf[m];
      qx[q] = (T)((float)p[0] * X + (float)p[1] * Y + (float)p[2] * Z);
      qx[capacity + q] = (T)((float)p[3] * X + (float)p[4] * Y + (float)p[5] * Z);
      qx[2 * capacity + q] = (T)((float)p[6] * X + (float)p[7] * Y + (float)p[8] * Z);
    }
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
                         long long total_nodes, T* __restrict__ out) {
  long long n = min(*d_count, capacity);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    int B = donor_grid[q];
    if (B < 0) continue;
    const GridDev& G = grids[B];
    int ci, cj, ck;
    cell_ijk(G, donor_cell[q], ci, cj, ck);
    T s0 = s[q], s1 = s[capacity + q], s2 = s[2 * capacity + q];
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
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const T* F = fields + (long long)f * total_nodes;
      T acc = 0;
#pragma unroll
      for (int c = 0; c < 8; ++c) acc += w[c] * F[nd[c]];
      out[(long long)f * capacity + q] = acc;
    }
  }
}

hipError_t launch_interp(ov_ctx* ctx, const int32_t* donor_grid, const int32_t* donor_cell, const void* s,
                         const long long* d_count, long long capacity, const void* fields, void* out, hipStream_t st) {
  int block = ctx->interp_block;
  long long grid = grid_size_for(ctx, capacity, block);
  long long total = ctx->node_off.back();
  if (ctx->precision == OV_MIXED)
    hipLaunchKernelGGL(k_interp<float>, dim3((unsigned)grid), dim3(block), 0, st, ctx->d_grids, donor_grid,
                       donor_cell, (const float*)s, d_count, capacity, (const float*)fields, total, (float*)out);
  else
    hipLaunchKernelGGL(k_interp<double>, dim3((unsigned)grid), dim3(block), 0, st, ctx->d_grids, donor_grid,
                       donor_cell, (const double*)s, d_count, capacity, (const double*)fields, total, (double*)out);
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
  hipError_t e = launch_fringe(ctx, nf, flags, s);
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
