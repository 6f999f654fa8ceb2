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
  double prm[kMaxGrids][3];
  double cull[kMaxGrids];
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
  for (int i = threadIdx.x; i < ngrids * 12; i += blockDim.x) L.pose[i / 12][i % 12] = poses[i];
  for (int g = threadIdx.x; g < ngrids; g += blockDim.x) {
    const GridDev& G = grids[g];
    L.off[g] = G.node_off;
    L.kind[g] = G.blank_kind;
    L.outer[g] = G.has_outer;
    L.cull[g] = G.cull_r2;
    L.prm[g][0] = G.blank_prm[0];
    L.prm[g][1] = G.blank_prm[1];
    L.prm[g][2] = G.blank_prm[2];
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

// Signed, scale-free inside measure of a body-frame point: < 0 strictly inside.
// For the cylinder the radial and axial conditions are combined as a max.
template <typename T>
__device__ __forceinline__ T blank_measure(int kind, const double* prm, T x, T y, T z) {
  if (kind == OV_BLANK_SPHERE) {
    T r = (T)prm[0];
    return (x * x + y * y + z * z) / (r * r) - (T)1;
  }
  if (kind == OV_BLANK_ELLIPSOID) {
    T u = x / (T)prm[0], v = y / (T)prm[1], w = z / (T)prm[2];
    return u * u + v * v + w * w - (T)1;
  }
  // cylinder: inside iff rho^2 < r^2 and z0 <= z <= z1
  T r = (T)prm[0];
  T fr = (x * x + y * y) / (r * r) - (T)1;
  T fz = fmax(((T)prm[1] - z) / r, (z - (T)prm[2]) / r);
  return fmax(fr, fz);
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
  float w0 = (float)pa[0] * (float)X + (float)pa[1] * (float)Y + (float)pa[2] * (float)Z + (float)pa[9];
  float w1 = (float)pa[3] * (float)X + (float)pa[4] * (float)Y + (float)pa[5] * (float)Z + (float)pa[10];
  float w2 = (float)pa[6] * (float)X + (float)pa[7] * (float)Y + (float)pa[8] * (float)Z + (float)pa[11];
  bool unsure = false;
  int cause = -1;
  for (int b = 0; b < L.nblank; ++b) {
    int B = L.blank[b];
    if (B == A) continue;
    const double* p = L.pose[B];
    float d0 = w0 - (float)p[9], d1 = w1 - (float)p[10], d2 = w2 - (float)p[11];
    if (d0 * d0 + d1 * d1 + d2 * d2 >= (float)L.cull[B] * 1.0001f + 1e-30f) continue;
    float x = (float)p[0] * d0 + (float)p[3] * d1 + (float)p[6] * d2;
    float y = (float)p[1] * d0 + (float)p[4] * d1 + (float)p[7] * d2;
    float z = (float)p[2] * d0 + (float)p[5] * d1 + (float)p[8] * d2;
    float f = blank_measure<float>(L.kind[B], L.prm[B], x, y, z);
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
__device__ __forceinline__ uint8_t node_flag(const GridDev& G, long long m, int cause, uint8_t* tile_hole) {
  if (cause < 0 && !G.has_outer) return (uint8_t)OV_STATE_FIELD;
  long long plane = (long long)G.ni * G.nj;
  int k = (int)(m / plane);
  long long r = m - (long long)k * plane;
  int j = (int)(r / G.ni);
  int i = (int)(r - (long long)j * G.ni);
  if (cause >= 0) {
    tile_hole[G.tile_off + (i >> 6) + (long long)G.tiles_i * ((j >> 3) + (long long)G.tiles_j * (k >> 3))] = 1;
    return (uint8_t)(kHole | (cause << 2));
  }
  bool onb = i < G.outer[0] || i >= G.ni - G.outer[1] || j < G.outer[2] || j >= G.nj - G.outer[3] ||
             k < G.outer[4] || k >= G.nk - G.outer[5];
  return onb ? (uint8_t)(kFringe | (OV_CAUSE_BOUNDARY << 2)) : (uint8_t)OV_STATE_FIELD;
}

template <typename CT, int NPT>
__global__ void __launch_bounds__(1024) k_holecut(const GridDev* __restrict__ grids, int ngrids,
                                                 const double* __restrict__ poses, uint8_t* __restrict__ flags,
                                                 long long total, uint8_t* __restrict__ tile_hole) {
  __shared__ HoleLds L;
  holecut_stage<CT>(L, grids, ngrids, poses);
  const long long span = (long long)blockDim.x * NPT;
  for (long long base = (long long)blockIdx.x * span; base < total; base += (long long)gridDim.x * span) {
    CT X[NPT], Y[NPT], Z[NPT];
    int A[NPT];
    long long m[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      long long n = base + (long long)r * blockDim.x + threadIdx.x;
      A[r] = 0;
      m[r] = -1;
      if (n < total) {
        A[r] = grid_of_node(L.off, ngrids, n);
        m[r] = n - L.off[A[r]];
        X[r] = __builtin_nontemporal_load((const CT*)L.X[A[r]] + m[r]);
        Y[r] = __builtin_nontemporal_load((const CT*)L.Y[A[r]] + m[r]);
        Z[r] = __builtin_nontemporal_load((const CT*)L.Z[A[r]] + m[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      if (m[r] < 0) continue;
      int cause = holecut_node<CT>(L, grids, A[r], m[r], X[r], Y[r], Z[r]);
      flags[base + (long long)r * blockDim.x + threadIdx.x] =
          (cause < 0 && !L.outer[A[r]]) ? (uint8_t)OV_STATE_FIELD : node_flag(grids[A[r]], m[r], cause, tile_hole);
    }
  }
}

template <typename CT>
static void launch_holecut_t(ov_ctx* ctx, const double* poses, uint8_t* flags, hipStream_t s) {
  long long total = ctx->node_off.back();
  int block = ctx->holecut_block;
  int npt = ctx->holecut_npt;
  long long chunks = (total + (long long)block * npt - 1) / ((long long)block * npt);
  int per_cu = ctx->persist > 0 ? ctx->persist : 8;
  long long grid = std::max(1LL, std::min(chunks, (long long)ctx->num_cus * per_cu));
  int ng = (int)ctx->grids.size();
  if (npt == 4)
    hipLaunchKernelGGL((k_holecut<CT, 4>), dim3((unsigned)grid), dim3(block), 0, s, ctx->d_grids, ng, poses, flags,
                       total, ctx->d_tile_hole);
  else if (npt == 2)
    hipLaunchKernelGGL((k_holecut<CT, 2>), dim3((unsigned)grid), dim3(block), 0, s, ctx->d_grids, ng, poses, flags,
                       total, ctx->d_tile_hole);
  else
    hipLaunchKernelGGL((k_holecut<CT, 1>), dim3((unsigned)grid), dim3(block), 0, s, ctx->d_grids, ng, poses, flags,
                       total, ctx->d_tile_hole);
}

hipError_t launch_holecut(ov_ctx* ctx, const double* poses, uint8_t* flags, hipStream_t s) {
  if (ctx->precision == OV_MIXED) launch_holecut_t<float>(ctx, poses, flags, s);
  else launch_holecut_t<double>(ctx, poses, flags, s);
  return hipGetLastError();
}

// ================================================================ fringe marking
// The hole cut already wrote holes, the outer-boundary layers and, per 3D
// tile of kTileI x kTileJ x kTileK nodes, whether the tile holds a hole.
// Only tiles with a hole in themselves or a neighbour tile (nf < tile size,
// so the buffer reaches no further) can gain buffer nodes: one thread per
// tile lists them, then one block per listed tile stages the tile plus an
// nf halo in LDS as "cause if hole, 255 otherwise" and takes the lowest cause
// within Chebyshev distance nf by a separable min filter (i, then j, then k).
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

__global__ void __launch_bounds__(256) k_fringe_near(const GridDev* __restrict__ grids, int ngrids,
                                                    const uint8_t* __restrict__ tile_hole, long long total_tiles,
                                                    int* __restrict__ near_list, int* __restrict__ near_count) {
  for (long long tile = (long long)blockIdx.x * blockDim.x + threadIdx.x; tile < total_tiles;
       tile += (long long)gridDim.x * blockDim.x) {
    const GridDev& G = grids[tile_grid(grids, ngrids, tile)];
    int ti, tj, tk;
    tile_coords(G, tile, ti, tj, tk);
    bool near = false;
    for (int dz = -1; dz <= 1 && !near; ++dz) {
      int z = wrap_or_out(tk + dz, G.tiles_k, G.per & 4);
      if (z < 0) continue;
      for (int dy = -1; dy <= 1 && !near; ++dy) {
        int y = wrap_or_out(tj + dy, G.tiles_j, G.per & 2);
        if (y < 0) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          int x = wrap_or_out(ti + dx, G.tiles_i, G.per & 1);
          if (x < 0) continue;
          if (tile_hole[G.tile_off + x + (long long)G.tiles_i * (y + (long long)G.tiles_j * z)]) {
            near = true;
            break;
          }
        }
      }
    }
    if (near) {
      int slot = atomicAdd(near_count, 1);
      if ((long long)slot < total_tiles) near_list[slot] = (int)tile;
    }
  }
}

template <int NF>
__global__ void __launch_bounds__(256) k_fringe_tiles(const GridDev* __restrict__ grids, int ngrids,
                                                     uint8_t* __restrict__ flags, const int* __restrict__ near_list,
                                                     const int* __restrict__ near_count, long long total_tiles) {
  constexpr int EI = kTileI + 2 * NF, EJ = kTileJ + 2 * NF, EK = kTileK + 2 * NF;
  __shared__ uint8_t a[EK][EJ][EI];
  __shared__ uint8_t b[EK][EJ][kTileI];
  __shared__ uint8_t c[EK][kTileJ][kTileI];
  const long long nnear = min((long long)*near_count, total_tiles);
  for (long long it = blockIdx.x; it < nnear; it += gridDim.x) {
    const long long tile = near_list[it];
    const GridDev& G = grids[tile_grid(grids, ngrids, tile)];
    int ti, tj, tk;
    tile_coords(G, tile, ti, tj, tk);
    const int i0 = ti * kTileI, j0 = tj * kTileJ, k0 = tk * kTileK;
    uint8_t* fl = flags + G.node_off;
    for (int e = threadIdx.x; e < EI * EJ * EK; e += blockDim.x) {
      int x = e % EI, y = (e / EI) % EJ, z = e / (EI * EJ);
      int i = wrap_or_out(i0 - NF + x, G.ni, G.per & 1);
      int j = wrap_or_out(j0 - NF + y, G.nj, G.per & 2);
      int k = wrap_or_out(k0 - NF + z, G.nk, G.per & 4);
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
      uint8_t cause = 255;
#pragma unroll
      for (int d = 0; d <= 2 * NF; ++d) cause = min(cause, c[z + d][y][x]);
      if (cause == 255) continue;
      long long m = (long long)i + (long long)G.ni * ((long long)j + (long long)G.nj * k);
      // buffer causes are grid ids < 63, so they win over an outer-boundary cause
      if ((fl[m] & 3) != kHole) fl[m] = (uint8_t)(kFringe | (cause << 2));
    }
    __syncthreads();
  }
}

hipError_t launch_fringe(ov_ctx* ctx, int nf, uint8_t* flags, hipStream_t s) {
  if (nf == 0) return hipSuccess;  // outer layers were marked by the hole cut
  const int ng = (int)ctx->grids.size();
  long long g1 = std::max(1LL, std::min<long long>((ctx->total_tiles + 255) / 256, 65535));
  hipLaunchKernelGGL(k_fringe_near, dim3((unsigned)g1), dim3(256), 0, s, ctx->d_grids, ng, ctx->d_tile_hole,
                     ctx->total_tiles, ctx->d_near_list, ctx->d_near_count);
  long long g2 = std::max(1LL, std::min<long long>(ctx->total_tiles, (long long)ctx->num_cus * 2));
  switch (nf) {
    case 1:
      hipLaunchKernelGGL(k_fringe_tiles<1>, dim3((unsigned)g2), dim3(256), 0, s, ctx->d_grids, ng, flags,
                         ctx->d_near_list, ctx->d_near_count, ctx->total_tiles);
      break;
    case 2:
      hipLaunchKernelGGL(k_fringe_tiles<2>, dim3((unsigned)g2), dim3(256), 0, s, ctx->d_grids, ng, flags,
                         ctx->d_near_list, ctx->d_near_count, ctx->total_tiles);
      break;
    default:
      hipLaunchKernelGGL(k_fringe_tiles<3>, dim3((unsigned)g2), dim3(256), 0, s, ctx->d_grids, ng, flags,
                         ctx->d_near_list, ctx->d_near_count, ctx->total_tiles);
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
                                                      long long capacity, int32_t* __restrict__ status,
                                                      int* __restrict__ near_count) {
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
    *near_count = 0;  // the fringe pass of this call has consumed its tile list
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
                     d_count, capacity, ctx->d_status, ctx->d_near_count);
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
