// Context management, grid registration and control-cell construction.
//
// Control cells follow Sec. 2.2.5 of the paper: an axis-aligned auxiliary
// Cartesian grid is laid over each donor grid (here over the grid's body
// frame, where it never moves) and each control cell lists the donor cells
// whose corner box reaches it. A point inside a donor cell is inside that
// cell's corner box, so the list of the point's control cell is complete:
// the brute-force fallback of the walk (Alg. 3) scans exactly that list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "ov_internal.h"

namespace ov {

int fail(ov_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

int hip_fail(ov_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, OV_EHIP, "%s: %s", what, hipGetErrorString(e));
}

long long grid_size_for(const ov_ctx* ctx, long long items, int block) {
  long long need = (items + block - 1) / block;
  if (need < 1) need = 1;
  if (ctx->persist > 0) {
    long long cap = (long long)ctx->num_cus * ctx->persist;
    if (need > cap) need = cap;
  }
  if (need > (1LL << 30)) need = 1LL << 30;
  return need;
}

// ---------------------------------------------------------------- setup kernels
// Per-block min/max of node coordinates (6 partials per block).
__global__ void k_bounds(const double* __restrict__ X, const double* __restrict__ Y,
                         const double* __restrict__ Z, long long n, double* __restrict__ part) {
  __shared__ double red[6][256];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x; m < n;
       m += (long long)gridDim.x * blockDim.x) {
    double v[3] = {X[m], Y[m], Z[m]};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], v[d]);
      hi[d] = fmax(hi[d], v[d]);
    }
  }
  for (int d = 0; d < 3; ++d) {
    red[d][threadIdx.x] = lo[d];
    red[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int d = 0; d < 3; ++d) {
        red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + w]);
        red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + w]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// pass 0: count entries per bin and the lowest cell per bin; pass 1: fill.
template <int PASS>
__global__ void k_bins(GridDev g, unsigned long long* __restrict__ cnt, int* __restrict__ rep,
                       const long long* __restrict__ start, int* __restrict__ cells) {
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < g.ncells;
       c += (long long)gridDim.x * blockDim.x) {
    double lo[3], hi[3];
    cell_box(g, c, lo, hi);
    int a0 = bin_axis(g, 0, lo[0]), a1 = bin_axis(g, 0, hi[0]);
    int b0 = bin_axis(g, 1, lo[1]), b1 = bin_axis(g, 1, hi[1]);
    int e0 = bin_axis(g, 2, lo[2]), e1 = bin_axis(g, 2, hi[2]);
    for (int z = e0; z <= e1; ++z)
      for (int y = b0; y <= b1; ++y)
        for (int x = a0; x <= a1; ++x) {
          long long b = x + (long long)g.nb[0] * (y + (long long)g.nb[1] * z);
          if (PASS == 0) {
            atomicAdd(&cnt[b], 1ULL);
          } else {
            unsigned long long p = atomicAdd(&cnt[b], 1ULL);
            cells[start[b] + (long long)p] = (int)c;
          }
        }
  }
}

// Sort each control cell's list by cell index (shell sort, one thread per
// control cell), so a scan in list order meets the lowest index first.
__global__ void k_bin_sort(const long long* __restrict__ start, int* __restrict__ cells, long long nbins) {
  const int gaps[8] = {701, 301, 132, 57, 23, 10, 4, 1};
  for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < nbins; b += (long long)gridDim.x * blockDim.x) {
    int* a = cells + start[b];
    const int n = (int)(start[b + 1] - start[b]);
    for (int gi = 0; gi < 8; ++gi) {
      const int gap = gaps[gi];
      for (int i = gap; i < n; ++i) {
        int v = a[i], j = i;
        while (j >= gap && a[j - gap] > v) {
          a[j] = a[j - gap];
          j -= gap;
        }
        a[j] = v;
      }
    }
  }
}

// Walk seed of each control cell: the listed donor cell whose corner mean is
// nearest the control cell's centre (ties: lowest index); -1 if none.
__global__ void k_bin_rep(GridDev g, const long long* __restrict__ start, const int* __restrict__ cells,
                          int* __restrict__ rep, long long nbins) {
  for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < nbins; b += (long long)gridDim.x * blockDim.x) {
    long long bx = b % g.nb[0], by = (b / g.nb[0]) % g.nb[1], bz = b / ((long long)g.nb[0] * g.nb[1]);
    double ctr[3] = {g.blo[0] + (bx + 0.5) / g.binv[0], g.blo[1] + (by + 0.5) / g.binv[1],
                     g.blo[2] + (bz + 0.5) / g.binv[2]};
    int best = -1;
    double bestd = INFINITY;
    for (long long e = start[b]; e < start[b + 1]; ++e) {
      int cell = cells[e];
      int ci, cj, ck;
      cell_ijk(g, cell, ci, cj, ck);
      double m[3] = {0.0, 0.0, 0.0};
      for (int c = 0; c < 8; ++c) {
        long long nd = corner_node(g, ci, cj, ck, c);
        m[0] += g.X[nd];
        m[1] += g.Y[nd];
        m[2] += g.Z[nd];
      }
      double d0 = m[0] * 0.125 - ctr[0], d1 = m[1] * 0.125 - ctr[1], d2 = m[2] * 0.125 - ctr[2];
      double d = d0 * d0 + d1 * d1 + d2 * d2;
      if (d < bestd || (d == bestd && cell < best)) {
        bestd = d;
        best = cell;
      }
    }
    rep[b] = best;
  }
}

// Sub-bin lists of the split control cells: one block per split bin, one
// thread per entry of its list; each cell goes on every sub-bin its padded
// box overlaps (the test that put it on the bin's list). PASS 0 counts,
// PASS 1 writes.
template <int PASS>
__global__ void k_subbins(GridDev g, const int* __restrict__ split, long long nsplit,
                          unsigned long long* __restrict__ cnt, const long long* __restrict__ sstart,
                          int* __restrict__ scells) {
  for (long long h = blockIdx.x; h < nsplit; h += gridDim.x) {
    const long long b = split[h];
    const int base = g.bsub[b];
    const int bx = (int)(b % g.nb[0]), by = (int)((b / g.nb[0]) % g.nb[1]),
              bz = (int)(b / ((long long)g.nb[0] * g.nb[1]));
    for (long long e = g.bstart[b] + threadIdx.x; e < g.bstart[b + 1]; e += blockDim.x) {
      const int c = g.bcells[e];
      double lo[3], hi[3];
      cell_box(g, c, lo, hi);
      const int x0 = sub_axis(g, 0, lo[0], bx), x1 = sub_axis(g, 0, hi[0], bx);
      const int y0 = sub_axis(g, 1, lo[1], by), y1 = sub_axis(g, 1, hi[1], by);
      const int z0 = sub_axis(g, 2, lo[2], bz), z1 = sub_axis(g, 2, hi[2], bz);
      for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y)
          for (int x = x0; x <= x1; ++x) {
            const long long k = base + x + kSubBins * (y + kSubBins * z);
            const unsigned long long p = atomicAdd(&cnt[k], 1ULL);
            if (PASS == 1) scells[sstart[k] + (long long)p] = c;
          }
    }
  }
}

// Bounding sphere (body frame) of each sub-tile (kSubI x kTileJ x kTileK
// nodes, kTileI / kSubI of them per tile along i, sub-tile sb of tile t at
// index t * kSubPerTile + sb): centre of its coordinate box, radius = half
// the box diagonal. A sub-tile past the grid's last node gets radius -inf
// (nothing reaches it).
__global__ void __launch_bounds__(256) k_tile_spheres(GridDev g, double4* __restrict__ out) {
  __shared__ double red[6][256];
  const long long nsub = (long long)g.tiles_i * g.tiles_j * g.tiles_k * kSubPerTile;
  constexpr int kSubNodes = kSubI * kTileJ * kTileK;
  for (long long u = blockIdx.x; u < nsub; u += gridDim.x) {
    const long long t = u / kSubPerTile;
    const int sb = (int)(u % kSubPerTile);
    int ti = (int)(t % g.tiles_i), tj = (int)((t / g.tiles_i) % g.tiles_j), tk = (int)(t / ((long long)g.tiles_i * g.tiles_j));
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int e = threadIdx.x; e < kSubNodes; e += blockDim.x) {
      int i = ti * kTileI + sb * kSubI + (e % kSubI), j = tj * kTileJ + (e / kSubI) % kTileJ,
          k = tk * kTileK + e / (kSubI * kTileJ);
      if (i >= g.ni || j >= g.nj || k >= g.nk) continue;
      long long m = (long long)i + (long long)g.ni * ((long long)j + (long long)g.nj * k);
      double v[3] = {g.X[m], g.Y[m], g.Z[m]};
      for (int d = 0; d < 3; ++d) {
        lo[d] = fmin(lo[d], v[d]);
        hi[d] = fmax(hi[d], v[d]);
      }
    }
    for (int d = 0; d < 3; ++d) {
      red[d][threadIdx.x] = lo[d];
      red[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w)
        for (int d = 0; d < 3; ++d) {
          red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + w]);
          red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + w]);
        }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (!(red[0][0] <= red[3][0])) {
        out[u] = make_double4(0.0, 0.0, 0.0, -INFINITY);  // no node
      } else {
        double c[3], r2 = 0.0;
        for (int d = 0; d < 3; ++d) {
          c[d] = 0.5 * (red[d][0] + red[3 + d][0]);
          double h = 0.5 * (red[3 + d][0] - red[d][0]);
          r2 += h * h;
        }
        out[u] = make_double4(c[0], c[1], c[2], sqrt(r2));
      }
    }
    __syncthreads();
  }
}

__global__ void k_fill_int(int* p, long long n, int v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u8(uint8_t* p, long long n, uint8_t v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u64(unsigned long long* p, long long n, unsigned long long v = 0ULL) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

static long long blocks_for(long long n, int block = 256) {
  long long b = (n + block - 1) / block;
  return std::max(1LL, std::min(b, 65536LL));
}

#define HIPCHK(expr, what)                       \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

int build_control_cells(ov_ctx* ctx, GridHost& gh, hipStream_t s) {
  GridDev& g = gh.d;
  // box of the nodes
  const int nbk = (int)std::min<long long>(1024, blocks_for(g.nnodes));
  double* d_part = nullptr;
  HIPCHK(hipMalloc(&d_part, sizeof(double) * 6 * nbk), "hipMalloc bounds");
  hipLaunchKernelGGL(k_bounds, dim3(nbk), dim3(256), 0, s, g.X, g.Y, g.Z, g.nnodes, d_part);
  std::vector<double> part(6 * nbk);
  HIPCHK(hipMemcpyAsync(part.data(), d_part, sizeof(double) * 6 * nbk, hipMemcpyDeviceToHost, s), "bounds copy");
  HIPCHK(hipStreamSynchronize(s), "bounds sync");
  (void)hipFree(d_part);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = 0; b < nbk; ++b)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], part[6 * b + d]);
      hi[d] = std::max(hi[d], part[6 * b + 3 + d]);
    }
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(lo[d]) || !std::isfinite(hi[d]))
      return fail(ctx, OV_EINVAL, "grid has non-finite coordinates");
  // about two donor cells per control cell along each axis, shaped after the box
  double ext[3], vol = 1.0;
  for (int d = 0; d < 3; ++d) {
    ext[d] = std::max(hi[d] - lo[d], 1e-300);
    vol *= ext[d];
  }
  double edge = std::cbrt(vol * 8.0 / (double)std::max(1LL, g.ncells));
  long long nbins = 1;
  for (int d = 0; d < 3; ++d) {
    int nb = (int)std::ceil(ext[d] / edge);
    nb = std::max(1, std::min(nb, 4096));
    g.nb[d] = nb;
    g.blo[d] = lo[d];
    g.bhi[d] = hi[d];
    g.binv[d] = nb / ext[d];
    nbins *= nb;
  }
  unsigned long long* d_cnt = nullptr;
  HIPCHK(hipMalloc(&d_cnt, sizeof(unsigned long long) * (nbins + 1)), "hipMalloc bin counts");
  HIPCHK(hipMalloc(&gh.brep, sizeof(int) * nbins), "hipMalloc bin rep");
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(nbins + 1)), dim3(256), 0, s, d_cnt, nbins + 1);
  hipLaunchKernelGGL(k_bins<0>, dim3(blocks_for(g.ncells)), dim3(256), 0, s, g, d_cnt, gh.brep,
                     (const long long*)nullptr, (int*)nullptr);
  std::vector<unsigned long long> cnt(nbins);
  HIPCHK(hipMemcpyAsync(cnt.data(), d_cnt, sizeof(unsigned long long) * nbins, hipMemcpyDeviceToHost, s),
         "bin count copy");
  HIPCHK(hipStreamSynchronize(s), "bin count sync");
  std::vector<long long> start(nbins + 1);
  start[0] = 0;
  for (long long b = 0; b < nbins; ++b) start[b + 1] = start[b] + (long long)cnt[b];
  long long entries = start[nbins];
  if (entries >= (1LL << 31)) {
    (void)hipFree(d_cnt);
    return fail(ctx, OV_EDIMS, "control-cell lists too large (%lld entries)", entries);
  }
  HIPCHK(hipMalloc(&gh.bstart, sizeof(long long) * (nbins + 1)), "hipMalloc bin start");
  HIPCHK(hipMalloc(&gh.bcells, sizeof(int) * std::max(1LL, entries)), "hipMalloc bin cells");
  HIPCHK(hipMemcpyAsync(gh.bstart, start.data(), sizeof(long long) * (nbins + 1), hipMemcpyHostToDevice, s),
         "bin start copy");
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(nbins + 1)), dim3(256), 0, s, d_cnt, nbins + 1);
  hipLaunchKernelGGL(k_bins<1>, dim3(blocks_for(g.ncells)), dim3(256), 0, s, g, d_cnt, (int*)nullptr,
                     (const long long*)gh.bstart, gh.bcells);
  HIPCHK(hipGetLastError(), "control-cell kernels");
  hipLaunchKernelGGL(k_bin_sort, dim3(blocks_for(nbins)), dim3(256), 0, s, (const long long*)gh.bstart, gh.bcells,
                     nbins);
  hipLaunchKernelGGL(k_bin_rep, dim3(blocks_for(nbins)), dim3(256), 0, s, g, (const long long*)gh.bstart,
                     (const int*)gh.bcells, gh.brep, nbins);
  HIPCHK(hipGetLastError(), "control-cell seeds");
  HIPCHK(hipStreamSynchronize(s), "control-cell sync");
  (void)hipFree(d_cnt);
  g.bstart = gh.bstart;
  g.bcells = gh.bcells;
  g.brep = gh.brep;
  g.bsub = nullptr;
  g.sstart = nullptr;
  g.scells = nullptr;
  return build_subbins(ctx, gh, cnt, s);
}

// Second level of the control cells: bins listing more than kSplitList
// cells (where cells are much smaller than a bin, e.g. the wedge cells of a
// shell around its polar axis) get kSubBins^3 sub-bins, so that the
// brute-force scan of a point reads one sub-bin's list.
int build_subbins(ov_ctx* ctx, GridHost& gh, const std::vector<unsigned long long>& cnt, hipStream_t s) {
  GridDev& g = gh.d;
  const long long nbins = (long long)cnt.size();
  std::vector<int> split, bsub(nbins, -1);
  constexpr long long per = (long long)kSubBins * kSubBins * kSubBins;
  for (long long b = 0; b < nbins; ++b)
    if ((long long)cnt[b] > kSplitList) {
      bsub[b] = (int)(per * (long long)split.size());
      split.push_back((int)b);
    }
  if (split.empty()) return OV_OK;
  const long long nsplit = (long long)split.size(), nsub = per * nsplit;
  if (nsub >= (1LL << 31)) return fail(ctx, OV_EDIMS, "too many split control cells");
  int* d_split = nullptr;
  unsigned long long* d_cnt = nullptr;
  HIPCHK(hipMalloc(&gh.bsub, sizeof(int) * nbins), "hipMalloc sub-bin index");
  HIPCHK(hipMalloc(&d_split, sizeof(int) * nsplit), "hipMalloc split bins");
  HIPCHK(hipMalloc(&d_cnt, sizeof(unsigned long long) * (nsub + 1)), "hipMalloc sub-bin counts");
  HIPCHK(hipMemcpyAsync(gh.bsub, bsub.data(), sizeof(int) * nbins, hipMemcpyHostToDevice, s), "sub-bin index copy");
  HIPCHK(hipMemcpyAsync(d_split, split.data(), sizeof(int) * nsplit, hipMemcpyHostToDevice, s), "split bins copy");
  g.bsub = gh.bsub;
  const unsigned nblk = (unsigned)std::min<long long>(nsplit, 65536);
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(nsub + 1)), dim3(256), 0, s, d_cnt, nsub + 1);
  hipLaunchKernelGGL(k_subbins<0>, dim3(nblk), dim3(256), 0, s, g, (const int*)d_split, nsplit, d_cnt,
                     (const long long*)nullptr, (int*)nullptr);
  std::vector<unsigned long long> scnt(nsub);
  HIPCHK(hipMemcpyAsync(scnt.data(), d_cnt, sizeof(unsigned long long) * nsub, hipMemcpyDeviceToHost, s),
         "sub-bin count copy");
  HIPCHK(hipStreamSynchronize(s), "sub-bin count sync");
  std::vector<long long> start(nsub + 1);
  start[0] = 0;
  for (long long k = 0; k < nsub; ++k) start[k + 1] = start[k] + (long long)scnt[k];
  const long long entries = start[nsub];
  if (entries >= (1LL << 31)) {
    (void)hipFree(d_cnt);
    (void)hipFree(d_split);
    return fail(ctx, OV_EDIMS, "sub-bin lists too large (%lld entries)", entries);
  }
  HIPCHK(hipMalloc(&gh.sstart, sizeof(long long) * (nsub + 1)), "hipMalloc sub-bin start");
  HIPCHK(hipMalloc(&gh.scells, sizeof(int) * std::max(1LL, entries)), "hipMalloc sub-bin cells");
  HIPCHK(hipMemcpyAsync(gh.sstart, start.data(), sizeof(long long) * (nsub + 1), hipMemcpyHostToDevice, s),
         "sub-bin start copy");
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(nsub + 1)), dim3(256), 0, s, d_cnt, nsub + 1);
  hipLaunchKernelGGL(k_subbins<1>, dim3(nblk), dim3(256), 0, s, g, (const int*)d_split, nsplit, d_cnt,
                     (const long long*)gh.sstart, gh.scells);
  hipLaunchKernelGGL(k_bin_sort, dim3(blocks_for(nsub)), dim3(256), 0, s, (const long long*)gh.sstart, gh.scells,
                     nsub);
  HIPCHK(hipGetLastError(), "sub-bin kernels");
  HIPCHK(hipStreamSynchronize(s), "sub-bin sync");
  (void)hipFree(d_cnt);
  (void)hipFree(d_split);
  g.sstart = gh.sstart;
  g.scells = gh.scells;
  return OV_OK;
}

int build_shadows(ov_ctx* ctx, GridHost& gh, hipStream_t s) {
  GridDev& g = gh.d;
  HIPCHK(hipMalloc(&gh.xf, sizeof(float) * g.nnodes), "hipMalloc shadow");
  HIPCHK(hipMalloc(&gh.yf, sizeof(float) * g.nnodes), "hipMalloc shadow");
  HIPCHK(hipMalloc(&gh.zf, sizeof(float) * g.nnodes), "hipMalloc shadow");
  hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(g.nnodes)), dim3(256), 0, s, g.X, gh.xf, g.nnodes);
  hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(g.nnodes)), dim3(256), 0, s, g.Y, gh.yf, g.nnodes);
  hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(g.nnodes)), dim3(256), 0, s, g.Z, gh.zf, g.nnodes);
  HIPCHK(hipGetLastError(), "shadow kernels");
  g.Xf = gh.xf;
  g.Yf = gh.yf;
  g.Zf = gh.zf;
  return OV_OK;
}

// Whether the face at end `end` (0 low, 1 high) of axis `a` collapses onto
// lines along the periodic axis `pa`: every node of the face within `tol`
// (per component) of the face's node at periodic index 0 on the same line.
// *bad is set where one is not.
__global__ void k_face_collapsed(GridDev g, int a, int end, int pa, double tol, unsigned int* __restrict__ bad) {
  const int n[3] = {g.ni, g.nj, g.nk};
  const int q = 3 - a - pa;  // the face's other axis
  const long long cnt = (long long)n[pa] * n[q];
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < cnt;
       t += (long long)gridDim.x * blockDim.x) {
    int idx[3], ref[3];
    idx[a] = ref[a] = end ? n[a] - 1 : 0;
    idx[pa] = (int)(t % n[pa]);
    ref[pa] = 0;
    idx[q] = ref[q] = (int)(t / n[pa]);
    const long long m = idx[0] + (long long)g.ni * (idx[1] + (long long)g.nj * idx[2]);
    const long long r = ref[0] + (long long)g.ni * (ref[1] + (long long)g.nj * ref[2]);
    if (!(fabs(g.X[m] - g.X[r]) <= tol && fabs(g.Y[m] - g.Y[r]) <= tol && fabs(g.Z[m] - g.Z[r]) <= tol))
      atomicOr(bad, 1u);
  }
}

// The polar ends of a grid with one periodic axis (GridDev::pole): faces of
// the other two axes that collapse onto the axis of revolution, to within
// 1e-12 of the grid's extent.
static int find_poles(ov_ctx* ctx, GridHost& gh, hipStream_t s) {
  GridDev& g = gh.d;
  g.pole = 0;
  if (g.per != 1 && g.per != 2 && g.per != 4) return OV_OK;
  const int pa = g.per == 1 ? 0 : (g.per == 2 ? 1 : 2);
  double ext = 0.0;
  for (int d = 0; d < 3; ++d) ext = std::max(ext, g.bhi[d] - g.blo[d]);
  const double tol = 1e-12 * ext;
  unsigned int* d_bad = nullptr;
  HIPCHK(hipMalloc(&d_bad, sizeof(unsigned int) * 6), "hipMalloc pole test");
  hipError_t e = hipMemsetAsync(d_bad, 0, sizeof(unsigned int) * 6, s);
  const int n[3] = {g.ni, g.nj, g.nk};
  for (int a = 0; a < 3 && e == hipSuccess; ++a) {
    if (a == pa) continue;
    const long long cnt = (long long)n[pa] * n[3 - a - pa];
    for (int end = 0; end < 2; ++end)
      hipLaunchKernelGGL(k_face_collapsed, dim3(blocks_for(cnt)), dim3(256), 0, s, g, a, end, pa, tol,
                         d_bad + 2 * a + end);
  }
  unsigned int bad[6] = {1, 1, 1, 1, 1, 1};
  if (e == hipSuccess) e = hipMemcpyAsync(bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_bad);
  if (e != hipSuccess) return hip_fail(ctx, e, "pole test");
  for (int a = 0; a < 3; ++a)
    for (int end = 0; end < 2; ++end)
      if (a != pa && !bad[2 * a + end]) g.pole |= 1 << (2 * a + end);
  return OV_OK;
}

// Flags of a grid with outer-boundary layers before any hole cut: fringe
// (cause 63) on its outer layers, field elsewhere.
__global__ void k_base_flags(GridDev g, uint8_t* __restrict__ out) {
  for (long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x; m < g.nnodes;
       m += (long long)gridDim.x * blockDim.x) {
    const long long plane = (long long)g.ni * g.nj;
    const int k = (int)(m / plane);
    const long long r = m - (long long)k * plane;
    const int j = (int)(r / g.ni), i = (int)(r - (long long)j * g.ni);
    const bool on = i < g.outer[0] || i >= g.ni - g.outer[1] || j < g.outer[2] || j >= g.nj - g.outer[3] ||
                    k < g.outer[4] || k >= g.nk - g.outer[5];
    out[m] = on ? (uint8_t)(OV_STATE_FRINGE | (OV_CAUSE_BOUNDARY << 2)) : (uint8_t)OV_STATE_FIELD;
  }
}

__global__ void k_pack_xyz(const double* __restrict__ X, const double* __restrict__ Y, const double* __restrict__ Z,
                           long long n, double4* __restrict__ P) {
  for (long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x; m < n; m += (long long)gridDim.x * blockDim.x)
    P[m] = make_double4(X[m], Y[m], Z[m], 0.0);
}

__global__ void k_pack_xyz_f32(const double* __restrict__ X, const double* __restrict__ Y,
                               const double* __restrict__ Z, long long n, double ax, double ay, double az,
                               float4* __restrict__ P) {
  for (long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x; m < n; m += (long long)gridDim.x * blockDim.x)
    P[m] = make_float4((float)(X[m] - ax), (float)(Y[m] - ay), (float)(Z[m] - az), 0.0f);
}

// (x, y, z, 0) per node, 32 bytes: a cell's corners i and i+1 share a
// 64-byte span, so one cell is 4 row pairs instead of 12 separate lines of
// the three coordinate arrays. Built once: body-frame coordinates are fixed.
// Mixed precision adds the FP32 walk's copy, 16 bytes per node: offsets
// from the centre of the nodes' box, rounded to FP32. |offset| is at most
// the box's half extent h, so each component's rounding is at most 2^-24 h
// (round to nearest; the FP64 difference before it is exact to 2^-53).
int build_gather_layout(ov_ctx* ctx, GridHost& g, hipStream_t s) {
  HIPCHK(hipMalloc(&g.p, sizeof(double4) * g.d.nnodes), "hipMalloc gather layout");
  hipLaunchKernelGGL(k_pack_xyz, dim3(blocks_for(g.d.nnodes)), dim3(256), 0, s, g.d.X, g.d.Y, g.d.Z, g.d.nnodes,
                     g.p);
  HIPCHK(hipGetLastError(), "gather layout");
  g.d.P = g.p;
  g.d.PF = nullptr;
  g.d.pf_err = 0.0;
  if (ctx->precision == OV_MIXED) {
    double half = 0.0;
    for (int d = 0; d < 3; ++d) {
      g.d.anchor[d] = 0.5 * (g.d.blo[d] + g.d.bhi[d]);
      half = std::max(half, 0.5 * (g.d.bhi[d] - g.d.blo[d]));
    }
    g.d.pf_err = std::ldexp(half, -24) * (1.0 + 1e-6);
    HIPCHK(hipMalloc(&g.pf, sizeof(float4) * g.d.nnodes), "hipMalloc FP32 gather layout");
    hipLaunchKernelGGL(k_pack_xyz_f32, dim3(blocks_for(g.d.nnodes)), dim3(256), 0, s, g.d.X, g.d.Y, g.d.Z,
                       g.d.nnodes, g.d.anchor[0], g.d.anchor[1], g.d.anchor[2], g.pf);
    HIPCHK(hipGetLastError(), "FP32 gather layout");
    g.d.PF = g.pf;
  }
  return OV_OK;
}

}  // namespace ov

using namespace ov;

// ================================================================ C ABI
extern "C" {

int ov_ctx_create(ov_ctx** out, int device, int precision) {
  if (!out) return OV_EINVAL;
  *out = nullptr;
  if (precision != OV_FP64 && precision != OV_MIXED) return OV_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return OV_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return OV_EHIP;
  ov_ctx* ctx = new ov_ctx();
  ctx->device = device;
  ctx->precision = precision;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->num_cus = prop.multiProcessorCount;
  if (hipMalloc(&ctx->d_status, sizeof(int32_t)) != hipSuccess ||
      hipMemset(ctx->d_status, 0, sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&ctx->d_stats, sizeof(unsigned long long) * kStatSlots * kStatStride) != hipSuccess ||
      hipMemset(ctx->d_stats, 0, sizeof(unsigned long long) * kStatSlots * kStatStride) != hipSuccess) {
    delete ctx;
    return OV_EHIP;
  }
  // the no-allocation fringe call's static array on this device (without
  // it that one call refuses to run; nothing else depends on it)
  void* sp = nullptr;
  if (static_scratch_address(device, &sp) == hipSuccess) ctx->static_scratch = sp;
  *out = ctx;
  return OV_OK;
}

int ov_ctx_destroy(ov_ctx* ctx) {
  if (!ctx) return OV_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& g : ctx->grids) {
    (void)hipFree(g.xf);
    (void)hipFree(g.yf);
    (void)hipFree(g.zf);
    (void)hipFree(g.p);
    (void)hipFree(g.pf);
    (void)hipFree(g.bstart);
    (void)hipFree(g.bcells);
    (void)hipFree(g.brep);
    (void)hipFree(g.bsub);
    (void)hipFree(g.sstart);
    (void)hipFree(g.scells);
    (void)hipFree(g.mtri);
    (void)hipFree(g.mstart);
    (void)hipFree(g.mvox);
  }
  (void)hipFree(ctx->d_grids);
  (void)hipFree(ctx->d_status);
  (void)hipFree(ctx->d_stats);
  (void)hipFree(ctx->d_warm);
  (void)hipFree(ctx->d_tile_sphere);
  (void)hipFree(ctx->d_tile_info);
  (void)hipFree(ctx->d_base_flags);
  (void)hipFree(ctx->d_fill_ranges);
  (void)hipFree(ctx->d_stamp);
  (void)hipFree(ctx->d_tile_hole);
  (void)hipFree(ctx->d_sub_mask);
  (void)hipFree(ctx->d_mask_counts);
  (void)hipFree(ctx->d_tile_near);
  (void)hipFree(ctx->d_near_list);
  (void)hipFree(ctx->d_near_count);
  (void)hipFree(ctx->d_chunk_static);
  (void)hipFree(ctx->d_chunk_stamp);
  (void)hipFree(ctx->d_chunk_list);
  (void)hipFree(ctx->d_chunk_list_count);
  (void)hipFree(ctx->d_chunk_counts);
  (void)hipFree(ctx->d_super_counts);
  (void)hipFree(ctx->d_super_offsets);
  delete ctx;
  return OV_OK;
}

const char* ov_last_error(const ov_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ov_grid_add(ov_ctx* ctx, int32_t ni, int32_t nj, int32_t nk, uint32_t periodic, const double* X,
                const double* Y, const double* Z, int32_t blank_kind, const double* blank_prm,
                const int32_t* outer, int32_t* grid_id) {
  if (!ctx) return OV_EINVAL;
  if (ctx->finalized) return fail(ctx, OV_ESTATE, "ov_grid_add after ov_finalize");
  if (!X || !Y || !Z || !outer || !grid_id) return fail(ctx, OV_EINVAL, "null argument to ov_grid_add");
  if ((int)ctx->grids.size() >= kMaxGrids) return fail(ctx, OV_EINVAL, "at most %d grids", kMaxGrids);
  if (ni < 2 || nj < 2 || nk < 2) return fail(ctx, OV_EDIMS, "grid dims must be >= 2 (got %d %d %d)", ni, nj, nk);
  if (periodic > 7u) return fail(ctx, OV_EINVAL, "periodic mask must be in 0..7");
  if (blank_kind < OV_BLANK_NONE || blank_kind > OV_BLANK_ELLIPSOID)
    return fail(ctx, OV_EINVAL, "unknown blank kind %d", blank_kind);
  if (blank_kind != OV_BLANK_NONE && !blank_prm) return fail(ctx, OV_EINVAL, "blank parameters missing");
  long long n = (long long)ni * nj * nk;
  if (ctx->node_off.back() + n >= (1LL << 31)) return fail(ctx, OV_EDIMS, "total nodes must stay below 2^31");
  for (int f = 0; f < 6; ++f)
    if (outer[f] < 0 || outer[f] > 64) return fail(ctx, OV_EINVAL, "outer layers must be in 0..64");
  GridHost gh;
  GridDev& g = gh.d;
  g.ni = ni;
  g.nj = nj;
  g.nk = nk;
  g.per = (int)periodic;
  g.pole = 0;  // (found at ov_finalize)
  g.nci = (periodic & 1) ? ni : ni - 1;
  g.ncj = (periodic & 2) ? nj : nj - 1;
  g.nck = (periodic & 4) ? nk : nk - 1;
  g.nnodes = n;
  g.ncells = (long long)g.nci * g.ncj * g.nck;
  g.inv_nci = 1.0 / (double)g.nci;
  g.inv_plane = 1.0 / ((double)g.nci * (double)g.ncj);
  if (g.ncells >= (1LL << 31)) return fail(ctx, OV_EDIMS, "too many cells");
  g.node_off = ctx->node_off.back();
  g.X = X;
  g.Y = Y;
  g.Z = Z;
  g.blank_kind = blank_kind;
  double r2 = 0.0;
  if (blank_kind != OV_BLANK_NONE) {
    for (int p = 0; p < 8; ++p) g.blank_prm[p] = blank_prm[p];
    const double* q = blank_prm;
    if (blank_kind == OV_BLANK_CYL) {
      if (!(q[0] > 0) || !(q[2] >= q[1])) return fail(ctx, OV_EINVAL, "cylinder blank needs r > 0, z1 >= z0");
      double zm = std::max(std::fabs(q[1]), std::fabs(q[2]));
      r2 = q[0] * q[0] + zm * zm;
    } else if (blank_kind == OV_BLANK_SPHERE) {
      if (!(q[0] > 0)) return fail(ctx, OV_EINVAL, "sphere blank needs r > 0");
      r2 = q[0] * q[0];
    } else {
      if (!(q[0] > 0 && q[1] > 0 && q[2] > 0)) return fail(ctx, OV_EINVAL, "ellipsoid blank needs a, b, c > 0");
      double m = std::max(q[0], std::max(q[1], q[2]));
      r2 = m * m;
    }
  }
  // inflate so the cull never rejects a node the exact test would accept
  g.cull_r2 = r2 * (1.0 + 1e-9) + 1e-300;
  g.has_outer = 0;
  for (int f = 0; f < 6; ++f) {
    g.outer[f] = outer[f];
    if (outer[f] > 0) g.has_outer = 1;
  }
  g.tiles_i = (ni + kTileI - 1) / kTileI;
  g.tiles_j = (nj + kTileJ - 1) / kTileJ;
  g.tiles_k = (nk + kTileK - 1) / kTileK;
  g.tile_off = ctx->total_tiles;
  ctx->total_tiles += (long long)g.tiles_i * g.tiles_j * g.tiles_k;
  *grid_id = (int32_t)ctx->grids.size();
  ctx->grids.push_back(gh);
  ctx->node_off.push_back(g.node_off + n);
  return OV_OK;
}

int ov_grid_set_blank_mesh(ov_ctx* ctx, int32_t grid, const double* tri, int64_t ntri) {
  if (!ctx) return OV_EINVAL;
  if (ctx->finalized) return fail(ctx, OV_ESTATE, "ov_grid_set_blank_mesh after ov_finalize");
  if (grid < 0 || grid >= (int)ctx->grids.size()) return fail(ctx, OV_EINVAL, "no grid %d", grid);
  if (!tri || ntri < 4) return fail(ctx, OV_EINVAL, "a closed surface needs at least 4 triangles");
  if (ntri > (1LL << 28)) return fail(ctx, OV_EINVAL, "too many triangles");
  GridHost& g = ctx->grids[grid];
  double r2 = 0.0;
  for (long long k = 0; k < 9 * ntri; ++k)
    if (!std::isfinite(tri[k])) return fail(ctx, OV_EINVAL, "non-finite triangle coordinate");
  for (long long k = 0; k < 3 * ntri; ++k) {
    const double* v = tri + 3 * k;
    r2 = std::max(r2, v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  }
  g.mesh.assign(tri, tri + 9 * ntri);
  g.d.blank_kind = OV_BLANK_MESH;
  for (int p = 0; p < 8; ++p) g.d.blank_prm[p] = 0.0;
  // the surface lies in the ball through its farthest vertex; inflated as
  // for the implicit shapes
  g.d.cull_r2 = r2 * (1.0 + 1e-9) + 1e-300;
  return OV_OK;
}

// The (y, z) bins of a surface triangulation: 2 sqrt(n_tri) per axis (at
// most 512), so that a node meets few more triangles than the surface
// layers above it.
static int build_mesh_bins(ov_ctx* ctx, GridHost& g) {
  const long long ntri = (long long)g.mesh.size() / 9;
  const double* t = g.mesh.data();
  double* box = g.d.mbox;
  for (int d = 0; d < 3; ++d) {
    box[d] = INFINITY;
    box[3 + d] = -INFINITY;
  }
  for (long long k = 0; k < 3 * ntri; ++k)
    for (int d = 0; d < 3; ++d) {
      box[d] = std::min(box[d], t[3 * k + d]);
      box[3 + d] = std::max(box[3 + d], t[3 * k + d]);
    }
  const int n = (int)std::max(1.0, std::min(512.0, std::floor(2.0 * std::sqrt((double)ntri))));
  for (int a = 0; a < 2; ++a) {
    const double ext = box[4 + a] - box[1 + a];
    g.d.mn[a] = ext > 0.0 ? n : 1;
    g.d.minv[a] = ext > 0.0 ? n / ext : 0.0;
  }
  const int ny = g.d.mn[0], nz = g.d.mn[1];
  std::vector<int> start((size_t)ny * nz + 1, 0);
  auto range = [&](long long k, int& y0, int& y1, int& z0, int& z1) {
    const double* a = t + 9 * k;
    const double ylo = std::min(a[1], std::min(a[4], a[7])), yhi = std::max(a[1], std::max(a[4], a[7]));
    const double zlo = std::min(a[2], std::min(a[5], a[8])), zhi = std::max(a[2], std::max(a[5], a[8]));
    y0 = mesh_bin(ylo, box[1], g.d.minv[0], ny);
    y1 = mesh_bin(yhi, box[1], g.d.minv[0], ny);
    z0 = mesh_bin(zlo, box[2], g.d.minv[1], nz);
    z1 = mesh_bin(zhi, box[2], g.d.minv[1], nz);
  };
  for (long long k = 0; k < ntri; ++k) {
    int y0, y1, z0, z1;
    range(k, y0, y1, z0, z1);
    for (int z = z0; z <= z1; ++z)
      for (int y = y0; y <= y1; ++y) ++start[(size_t)z * ny + y + 1];
  }
  for (size_t b = 0; b < (size_t)ny * nz; ++b) start[b + 1] += start[b];
  // each bin's triangles stored contiguously, oriented counter-clockwise in
  // (y, z) by the same edge function the test uses; edge-on ones dropped
  std::vector<double> binned((size_t)start.back() * 9);
  std::vector<int> fill(start.begin(), start.end() - 1);
  for (long long k = 0; k < ntri; ++k) {
    const double* a = t + 9 * k;
    const double* b = a + 3;
    const double* c = a + 6;
    const double area = mesh_edge(a, b, c[1], c[2]);
    if (area == 0.0) continue;
    if (area < 0.0) std::swap(b, c);
    int y0, y1, z0, z1;
    range(k, y0, y1, z0, z1);
    for (int z = z0; z <= z1; ++z)
      for (int y = y0; y <= y1; ++y) {
        double* dst = binned.data() + 9 * (size_t)fill[(size_t)z * ny + y]++;
        for (int d = 0; d < 3; ++d) {
          dst[d] = a[d];
          dst[3 + d] = b[d];
          dst[6 + d] = c[d];
        }
      }
  }
  // (bins end where their fill stopped: edge-on triangles leave gaps at the
  // end of a bin, closed here)
  std::vector<int> st2(start.size(), 0);
  std::vector<double> packed;
  packed.reserve(binned.size());
  for (size_t bin = 0; bin + 1 < start.size(); ++bin) {
    st2[bin] = (int)(packed.size() / 9);
    packed.insert(packed.end(), binned.begin() + 9 * (size_t)start[bin], binned.begin() + 9 * (size_t)fill[bin]);
  }
  st2.back() = (int)(packed.size() / 9);
  if (packed.empty()) packed.assign(9, 0.0);
  HIPCHK(hipMalloc(&g.mtri, sizeof(double) * packed.size()), "hipMalloc surface triangles");
  HIPCHK(hipMemcpy(g.mtri, packed.data(), sizeof(double) * packed.size(), hipMemcpyHostToDevice),
         "surface triangles copy");
  HIPCHK(hipMalloc(&g.mstart, sizeof(int) * st2.size()), "hipMalloc surface bins");
  HIPCHK(hipMemcpy(g.mstart, st2.data(), sizeof(int) * st2.size(), hipMemcpyHostToDevice), "surface bins copy");
  g.d.mtri = g.mtri;
  g.d.mstart = g.mstart;
  // voxels: about 256 along the box's longest side. A voxel grown by 1e-4
  // of that side on every face is "the surface may pass" (status 2) when
  // some triangle can meet it: the voxel lies in the triangle's box and the
  // triangle's plane crosses it (two of the separating axes of a triangle
  // and a box; no voxel a triangle meets fails either). Every other voxel
  // takes the ray-parity status of its centre, which holds for every point
  // of the grown voxel (no surface there): also for a node whose FP32
  // body-frame position lies in the voxel (its FP32 error is far below the
  // growth)
  const double ext = std::max(box[3] - box[0], std::max(box[4] - box[1], box[5] - box[2]));
  const double h = ext / 256.0, pad = 1e-4 * ext;
  for (int d = 0; d < 3; ++d) {
    const double e = box[3 + d] - box[d];
    g.d.mvn[d] = e > 0.0 ? (int)std::min(256.0, std::max(1.0, std::ceil(e / h))) : 1;
    g.d.mvinv[d] = e > 0.0 ? g.d.mvn[d] / e : 0.0;
  }
  const int vx = g.d.mvn[0], vy = g.d.mvn[1], vz = g.d.mvn[2];
  std::vector<uint8_t> vox((size_t)vx * vy * vz, 0);
  for (long long k = 0; k < ntri; ++k) {
    const double* a = t + 9 * k;
    int r[3][2];
    for (int d = 0; d < 3; ++d) {
      const double lo = std::min(a[d], std::min(a[3 + d], a[6 + d])) - pad;
      const double hi = std::max(a[d], std::max(a[3 + d], a[6 + d])) + pad;
      r[d][0] = mesh_bin(lo, box[d], g.d.mvinv[d], g.d.mvn[d]);
      r[d][1] = mesh_bin(hi, box[d], g.d.mvinv[d], g.d.mvn[d]);
    }
    // the plane: unit normal; a voxel (half sizes e_d, grown by pad) meets
    // it iff |n . (centre - a)| <= sum_d |n_d| (e_d + pad)
    double nv[3] = {(a[4] - a[1]) * (a[8] - a[2]) - (a[5] - a[2]) * (a[7] - a[1]),
                    (a[5] - a[2]) * (a[6] - a[0]) - (a[3] - a[0]) * (a[8] - a[2]),
                    (a[3] - a[0]) * (a[7] - a[1]) - (a[4] - a[1]) * (a[6] - a[0])};
    const double nl = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    const bool plane = nl > 0.0 && std::isfinite(nl);
    double rad = 0.0;
    for (int d = 0; d < 3; ++d) {
      nv[d] = plane ? nv[d] / nl : 0.0;
      rad += std::fabs(nv[d]) * (0.5 / g.d.mvinv[d] + pad);
    }
    rad *= 1.0 + 1e-9;  // (rounding of the test itself)
    for (int z = r[2][0]; z <= r[2][1]; ++z)
      for (int y = r[1][0]; y <= r[1][1]; ++y)
        for (int x = r[0][0]; x <= r[0][1]; ++x) {
          if (plane) {
            const double cx = box[0] + (x + 0.5) / g.d.mvinv[0], cy = box[1] + (y + 0.5) / g.d.mvinv[1],
                         cz = box[2] + (z + 0.5) / g.d.mvinv[2];
            if (std::fabs(nv[0] * (cx - a[0]) + nv[1] * (cy - a[1]) + nv[2] * (cz - a[2])) > rad) continue;
          }
          vox[((size_t)z * vy + y) * vx + x] = 2;
        }
  }
  for (int z = 0; z < vz; ++z)
    for (int y = 0; y < vy; ++y)
      for (int x = 0; x < vx; ++x) {
        uint8_t& v = vox[((size_t)z * vy + y) * vx + x];
        if (v == 2) continue;
        const double cx = box[0] + (x + 0.5) / g.d.mvinv[0], cy = box[1] + (y + 0.5) / g.d.mvinv[1],
                     cz = box[2] + (z + 0.5) / g.d.mvinv[2];
        v = mesh_parity(packed.data(), st2.data(), box, g.d.minv, g.d.mn, cx, cy, cz) ? 1 : 0;
      }
  HIPCHK(hipMalloc(&g.mvox, vox.size()), "hipMalloc surface voxels");
  HIPCHK(hipMemcpy(g.mvox, vox.data(), vox.size(), hipMemcpyHostToDevice), "surface voxels copy");
  g.d.mvox = g.mvox;
  return OV_OK;
}

int ov_finalize(ov_ctx* ctx, void* stream) {
  if (!ctx) return OV_EINVAL;
  if (ctx->finalized) return fail(ctx, OV_ESTATE, "already finalized");
  if (ctx->grids.empty()) return fail(ctx, OV_ESTATE, "no grids");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  for (auto& g : ctx->grids) {
    int rc = build_control_cells(ctx, g, s);
    if (rc == OV_OK) rc = find_poles(ctx, g, s);
    if (rc != OV_OK) return rc;
    if (ctx->precision == OV_MIXED) {
      rc = build_shadows(ctx, g, s);
      if (rc != OV_OK) return rc;
    }
    rc = build_gather_layout(ctx, g, s);
    if (rc != OV_OK) return rc;
    if (g.d.blank_kind == OV_BLANK_MESH) {
      rc = build_mesh_bins(ctx, g);
      if (rc != OV_OK) return rc;
      ctx->has_mesh = true;
    }
  }
  long long total = ctx->node_off.back();
  std::vector<GridDev> table;
  for (auto& g : ctx->grids) table.push_back(g.d);
  HIPCHK(hipMalloc(&ctx->d_grids, sizeof(GridDev) * table.size()), "hipMalloc grid table");
  HIPCHK(hipMemcpy(ctx->d_grids, table.data(), sizeof(GridDev) * table.size(), hipMemcpyHostToDevice),
         "grid table copy");
  HIPCHK(hipMalloc(&ctx->d_warm, sizeof(unsigned long long) * total), "hipMalloc warm-start records");
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(total)), dim3(256), 0, s, ctx->d_warm, total, kWarmEmpty);
  HIPCHK(hipMalloc(&ctx->d_tile_sphere, sizeof(double4) * kSubPerTile * std::max(1LL, ctx->total_tiles)),
         "hipMalloc sub-tile spheres");
  for (auto& g : ctx->grids) {
    long long nsub = (long long)g.d.tiles_i * g.d.tiles_j * g.d.tiles_k * kSubPerTile;
    hipLaunchKernelGGL(k_tile_spheres, dim3((unsigned)std::min(nsub, 65536LL)), dim3(256), 0, s, g.d,
                       ctx->d_tile_sphere + g.d.tile_off * kSubPerTile);
  }
  // front-half scratch (stamps start at 0: "never listed")
  const long long nt = std::max(1LL, ctx->total_tiles);
  {
    // the hole cut visits sub-tile (idx * sub_perm) mod nsub at position idx:
    // a prime near nsub / golden ratio that does not divide nsub is prime to
    // it, and keeps neighbouring sub-tiles far apart in the visiting order
    const long long nsub = nt * kSubPerTile;
    auto is_prime = [](long long v) {
      if (v < 2) return false;
      for (long long d = 2; d * d <= v; ++d)
        if (v % d == 0) return false;
      return true;
    };
    ctx->sub_perm = 1;
    if (nsub > 2 && nsub < (1LL << 31))
      for (long long p = (long long)(0.6180339887 * (double)nsub); p > 1; --p)
        if (is_prime(p) && nsub % p != 0) {
          ctx->sub_perm = p;
          break;
        }
  }
  {
    std::vector<int4> info((size_t)nt, make_int4(0, 0, 0, 0));
    for (size_t gi = 0; gi < ctx->grids.size(); ++gi) {
      const GridDev& g = ctx->grids[gi].d;
      for (int tk = 0; tk < g.tiles_k; ++tk)
        for (int tj = 0; tj < g.tiles_j; ++tj)
          for (int ti = 0; ti < g.tiles_i; ++ti)
            info[(size_t)(g.tile_off + ti + (long long)g.tiles_i * (tj + (long long)g.tiles_j * tk))] =
                make_int4((int)gi, ti, tj, tk);
    }
    HIPCHK(hipMalloc(&ctx->d_tile_info, sizeof(int4) * nt), "hipMalloc tile info");
    HIPCHK(hipMemcpy(ctx->d_tile_info, info.data(), sizeof(int4) * nt, hipMemcpyHostToDevice), "tile info copy");
    // fill ranges: consecutive grids with (kind 1) or without (kind 0) outer layers
    std::vector<long long> ranges;
    long long words = 0;
    for (size_t gi = 0; gi < ctx->grids.size(); ++gi) {
      const GridDev& g = ctx->grids[gi].d;
      const long long kind = g.has_outer ? 1 : 0;
      const long long a = g.node_off, b = g.node_off + g.nnodes;
      if (!ranges.empty() && ranges[ranges.size() - 1] == kind && ranges[ranges.size() - 3] == a) {
        ranges[ranges.size() - 3] = b;  // extend the previous range
      } else {
        ranges.push_back(a);
        ranges.push_back(b);
        ranges.push_back(0);
        ranges.push_back(kind);
      }
    }
    ctx->n_fill_ranges = (int)(ranges.size() / 4);
    for (int r = 0; r < ctx->n_fill_ranges; ++r) {
      const long long a = ranges[4 * r], b = ranges[4 * r + 1];
      ranges[4 * r + 2] = words;
      const long long wa = (a + 15) / 16, wb = b / 16;
      words += wb > wa ? wb - wa : 0;
    }
    ctx->fill_words = words;
    HIPCHK(hipMalloc(&ctx->d_base_flags, std::max(1LL, total)), "hipMalloc base flags");
    for (auto& g : ctx->grids)
      if (g.d.has_outer)
        hipLaunchKernelGGL(k_base_flags, dim3(blocks_for(g.d.nnodes)), dim3(256), 0, s, g.d,
                           ctx->d_base_flags + g.d.node_off);
    HIPCHK(hipGetLastError(), "base flags");
    HIPCHK(hipMalloc(&ctx->d_fill_ranges, sizeof(long long) * ranges.size()), "hipMalloc fill ranges");
    HIPCHK(hipMemcpy(ctx->d_fill_ranges, ranges.data(), sizeof(long long) * ranges.size(), hipMemcpyHostToDevice),
           "fill ranges copy");
  }
  HIPCHK(hipMalloc(&ctx->d_stamp, sizeof(unsigned int) * (2 + kSlots)), "hipMalloc stamps");
  HIPCHK(hipMalloc(&ctx->d_tile_hole, sizeof(unsigned int) * kSlots * nt), "hipMalloc tile holes");
  ctx->nmask_chunks = (nt * kSubPerTile + kMaskChunk - 1) / kMaskChunk;
  HIPCHK(hipMalloc(&ctx->d_sub_mask, sizeof(unsigned long long) * kSlots * kSubPerTile * nt), "hipMalloc sub-tile masks");
  HIPCHK(hipMalloc(&ctx->d_mask_counts, sizeof(int32_t) * kSlots * ctx->nmask_chunks), "hipMalloc mask counts");
  HIPCHK(hipMalloc(&ctx->d_tile_near, sizeof(unsigned int) * kSlots * nt), "hipMalloc tile near");
  // two near lists per slot (alternate steps of a slot write one each)
  HIPCHK(hipMalloc(&ctx->d_near_list, sizeof(int4) * 2 * kSlots * nt), "hipMalloc near lists");
  HIPCHK(hipMalloc(&ctx->d_near_count, sizeof(int32_t) * 2 * kSlots), "hipMalloc near counts");
  HIPCHK(hipMemsetAsync(ctx->d_stamp, 0, sizeof(unsigned int) * (2 + kSlots), s), "stamp init");
  HIPCHK(hipMemsetAsync(ctx->d_tile_hole, 0, sizeof(unsigned int) * kSlots * nt, s), "tile hole init");
  HIPCHK(hipMemsetAsync(ctx->d_tile_near, 0, sizeof(unsigned int) * kSlots * nt, s), "tile near init");
  HIPCHK(hipMemsetAsync(ctx->d_near_count, 0, sizeof(int32_t) * 2 * kSlots, s), "near count init");
  ctx->nchunks = (total + kCompactChunk - 1) / kCompactChunk;
  ctx->nsuper = (ctx->nchunks + kSuperChunk - 1) / kSuperChunk;
  HIPCHK(hipMalloc(&ctx->d_chunk_static, ctx->nchunks), "hipMalloc static chunk marks");
  // the fringe pass's and the compaction's chunk records, one set per
  // scratch slot: the steps of different slots may run them at once
  HIPCHK(hipMalloc(&ctx->d_chunk_stamp, sizeof(unsigned int) * kSlots * ctx->nchunks), "hipMalloc chunk stamps");
  HIPCHK(hipMalloc(&ctx->d_chunk_list, sizeof(int32_t) * kSlots * ctx->nchunks), "hipMalloc chunk list");
  HIPCHK(hipMalloc(&ctx->d_chunk_list_count, sizeof(int32_t) * kSlots), "hipMalloc chunk list counts");
  HIPCHK(hipMalloc(&ctx->d_chunk_counts, sizeof(unsigned long long) * kSlots * ctx->nchunks),
         "hipMalloc chunk counts");
  HIPCHK(hipMalloc(&ctx->d_super_counts, sizeof(int32_t) * kSlots * kSuperSlots * ctx->nsuper),
         "hipMalloc superchunk counts");
  HIPCHK(hipMalloc(&ctx->d_super_offsets, sizeof(long long) * kSlots * (ctx->nsuper + 1)),
         "hipMalloc superchunk offsets");
  HIPCHK(hipMemsetAsync(ctx->d_chunk_stamp, 0, sizeof(unsigned int) * kSlots * ctx->nchunks, s), "chunk stamp init");
  HIPCHK(hipMemsetAsync(ctx->d_chunk_list_count, 0, sizeof(int32_t) * kSlots, s), "chunk list count init");
  HIPCHK(hipMemsetAsync(ctx->d_chunk_counts, 0, sizeof(unsigned long long) * kSlots * ctx->nchunks, s),
         "chunk count init");
  HIPCHK(hipMemsetAsync(ctx->d_super_counts, 0, sizeof(int32_t) * kSlots * kSuperSlots * ctx->nsuper, s),
         "superchunk count init");
  HIPCHK(hipGetLastError(), "finalize kernels");
  {
    int rc = build_static_chunks(ctx, s);
    if (rc != OV_OK) return rc;
  }
  HIPCHK(hipStreamSynchronize(s), "finalize sync");
  ctx->finalized = true;
  return OV_OK;
}

int32_t ov_num_grids(const ov_ctx* ctx) { return ctx ? (int32_t)ctx->grids.size() : 0; }
int64_t ov_total_nodes(const ov_ctx* ctx) { return ctx ? (int64_t)ctx->node_off.back() : 0; }

int ov_node_offsets(const ov_ctx* ctx, int64_t* out) {
  if (!ctx || !out) return OV_EINVAL;
  for (size_t g = 0; g < ctx->node_off.size(); ++g) out[g] = ctx->node_off[g];
  return OV_OK;
}

int ov_set_option(ov_ctx* ctx, int32_t key, int64_t v) {
  if (!ctx) return OV_EINVAL;
  auto block_ok = [](int64_t b) { return b >= 64 && b <= 1024 && b % 64 == 0; };
  switch (key) {
    case OV_OPT_WARM:
      if (v != 0 && v != 1) break;
      ctx->warm = (int)v;
      return OV_OK;
    case OV_OPT_MAX_WALK:
      if (v < 1 || v > 100000) break;
      ctx->max_walk = (int)v;
      return OV_OK;
    case OV_OPT_SEARCH_BLOCK:
      if (!block_ok(v) || v > 256) break;
      ctx->search_block = (int)v;
      return OV_OK;
    case OV_OPT_INTERP_BLOCK:
      if (!block_ok(v)) break;
      ctx->interp_block = (int)v;
      return OV_OK;
    case OV_OPT_HOLECUT_BLOCK:
      if (!block_ok(v)) break;
      ctx->holecut_block = (int)v;
      return OV_OK;
    case OV_OPT_HOLECUT_NPT:
      if (v != 1 && v != 2 && v != 4) break;
      ctx->holecut_npt = (int)v;
      return OV_OK;
    case OV_OPT_HOLECUT_CULL:
      if (v != 0 && v != 1) break;
      ctx->cull = (int)v;
      return OV_OK;
    case OV_OPT_HOLECUT_NPL:
      if (v != 4 && v != 16) break;
      ctx->holecut_npl = (int)v;
      return OV_OK;
    case OV_OPT_HOLECUT_LIST:
      if (v != 0 && v != 1) break;
      ctx->holecut_list = (int)v;
      return OV_OK;
    case OV_OPT_BACK_FUSED:
      if (v < 0 || v > 2) break;
      ctx->back_fused = (int)v;
      return OV_OK;
    case OV_OPT_BACK_BLOCKS:
      if (v < 1 || v > 32) break;
      ctx->back_blocks_per_cu = (int)v;
      return OV_OK;
    case OV_OPT_BACK_QUEUE:
      if (v != 0 && v != 1) break;
      ctx->back_queue = (int)v;
      return OV_OK;
    case OV_OPT_BACK_XCD:
      if (v < 0 || v > 64) break;
      ctx->back_xcd = (int)v;
      return OV_OK;
    case OV_OPT_BACK_BLOCK:
      if (v != 64 && v != 128 && v != 256) break;
      ctx->back_block = (int)v;
      return OV_OK;
    case OV_OPT_FIELD_LAYOUT:
      if (v != 0 && v != 1) break;
      ctx->field_layout = (int)v;
      return OV_OK;
    case OV_OPT_FRAME_VELOCITY:
      if (v != 0 && v != 1) break;
      ctx->frame_velocity = (int)v;
      return OV_OK;
    case OV_OPT_PERSIST:
      if (v < 0 || v > 32) break;
      ctx->persist = (int)v;
      return OV_OK;
    default:
      return fail(ctx, OV_EINVAL, "unknown option %d", key);
  }
  return fail(ctx, OV_EINVAL, "option %d: value %lld out of range", key, (long long)v);
}

int ov_reset_history(ov_ctx* ctx, void* stream) {
  if (!ctx) return OV_EINVAL;
  if (!ctx->finalized) return fail(ctx, OV_ESTATE, "ov_reset_history before ov_finalize");
  long long total = ctx->node_off.back();
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(total)), dim3(256), 0, (hipStream_t)stream, ctx->d_warm, total,
                     kWarmEmpty);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? OV_OK : hip_fail(ctx, e, "reset history");
}

int ov_status_fetch(ov_ctx* ctx, int32_t* host_status, void* stream) {
  if (!ctx || !host_status) return OV_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int32_t v = 0;
  hipError_t e = hipMemcpyAsync(&v, ctx->d_status, sizeof v, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->d_status, 0, sizeof(int32_t), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "status fetch");
  *host_status = v;
  return OV_OK;
}

int overset_status_fetch(ov_ctx* ctx, int32_t* host_status, void* stream) {
  return ov_status_fetch(ctx, host_status, stream);
}

const char* overset_last_error(const ov_ctx* ctx) { return ov_last_error(ctx); }

int ov_stats_fetch(ov_ctx* ctx, int64_t* host_out, void* stream) {
  if (!ctx || !host_out) return OV_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  static_assert(OV_STAT_COUNT <= kStatStride, "counters fit one slot");
  unsigned long long v[kStatSlots * kStatStride];
  hipError_t e = hipMemcpyAsync(v, ctx->d_stats, sizeof v, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->d_stats, 0, sizeof v, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "stats fetch");
  for (int i = 0; i < OV_STAT_COUNT; ++i) {
    unsigned long long sum = 0;
    for (int k = 0; k < kStatSlots; ++k) sum += v[k * kStatStride + i];
    host_out[i] = (int64_t)sum;
  }
  return OV_OK;
}

}  // extern "C"
