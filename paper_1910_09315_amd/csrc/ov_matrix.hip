// Velocities in the receiver's frame (Sec. 2.3 of arXiv:1910.09315) and the
// interpolation matrix with its repeated application (Sec. 2.2.6, second
// option; Alg. 4).
//
// Frame velocity: a velocity interpolated from donor grid B has components
// in B's non-inertial frame; with poses x = R X + c (R = Q^T of the paper),
// the receiver, a node of grid A, gets u_A = R_A^T R_B u_B. Formed in FP64.
//
// Matrix: one ELL row of 8 entries per query (row-major, so a row is two
// 16-byte loads of indices and two or four of weights): the global index of
// each corner of the donor cell (grids packed by node offset: the paper's
// global index on one GPU) and its trilinear weight. The application
// y = M x for nrhs field vectors reads each row once and gathers its 8
// columns from every vector: the product the implicit solver repeats at
// every Newton-Krylov iteration.
#include <hip/hip_runtime.h>

#include "ov_internal.h"

namespace ov {

template <typename T>
__global__ void k_frame_velocity(const double* __restrict__ poses, const int32_t* __restrict__ q_grid,
                                 const int32_t* __restrict__ donor_grid, const long long* __restrict__ d_count,
                                 long long capacity, T* __restrict__ out) {
  const long long n = min(*d_count, capacity);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    const int B = donor_grid[q];
    if (B < 0) continue;
    T v[3] = {out[q], out[capacity + q], out[2 * capacity + q]};
    frame_rotate<T>(poses + 12 * q_grid[q], poses + 12 * B, v);
    out[q] = v[0];
    out[capacity + q] = v[1];
    out[2 * capacity + q] = v[2];
  }
}

hipError_t launch_frame_velocity(ov_ctx* ctx, const double* poses, const int32_t* q_grid,
                                 const int32_t* donor_grid, const long long* d_count, long long capacity, void* out,
                                 hipStream_t st) {
  const long long grid = grid_size_for(ctx, capacity, 256);
  if (ctx->precision == OV_MIXED)
    hipLaunchKernelGGL(k_frame_velocity<float>, dim3((unsigned)grid), dim3(256), 0, st, poses, q_grid, donor_grid,
                       d_count, capacity, (float*)out);
  else
    hipLaunchKernelGGL(k_frame_velocity<double>, dim3((unsigned)grid), dim3(256), 0, st, poses, q_grid, donor_grid,
                       d_count, capacity, (double*)out);
  return hipGetLastError();
}

template <typename T>
__global__ void k_interp_matrix(const GridDev* __restrict__ grids, const int32_t* __restrict__ donor_grid,
                                const int32_t* __restrict__ donor_cell, const T* __restrict__ s,
                                const long long* __restrict__ d_count, long long capacity,
                                int32_t* __restrict__ cols, T* __restrict__ vals) {
  const long long n = min(*d_count, capacity);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    const int B = donor_grid[q];
    int c8[8];
    T w8[8];
    if (B < 0) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        c8[c] = -1;
        w8[c] = (T)0;
      }
    } else {
      const GridDev& G = grids[B];
      int ci, cj, ck;
      cell_ijk(G, donor_cell[q], ci, cj, ck);
      const T s0 = s[q], s1 = s[capacity + q], s2 = s[2 * capacity + q];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const T a = (c & 1) ? s0 : (T)1 - s0;
        const T b = (c & 2) ? s1 : (T)1 - s1;
        const T d = (c & 4) ? s2 : (T)1 - s2;
        w8[c] = a * b * d;
        c8[c] = (int32_t)(G.node_off + corner_node(G, ci, cj, ck, c));
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      cols[8 * q + c] = c8[c];
      vals[8 * q + c] = w8[c];
    }
  }
}

// One row per thread: its 8 indices and weights as two 16-byte loads each
// (fp32) or two and four (fp64), then for each vector the 8 gathered values,
// summed in corner order. Vectors as blocks (x[r*total + node],
// y[r*capacity + row]) or interleaved (x[node*nrhs + r], y[row*nrhs + r]);
// interleaved with NR = 4 gathers each corner's 4 values with one load and
// writes the row's 4 results with one store. NR = 0: nrhs at run time.
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  typedef ov_fv4 type;
};
template <>
struct Vec4<double> {
  typedef double type __attribute__((ext_vector_type(4)));
};

template <typename T>
__device__ __forceinline__ void load_row(const int32_t* cols, const T* vals, long long q, int c8[8], T w8[8]) {
  gmem<ov_iv4>* cp = (gmem<ov_iv4>*)(gp(cols) + 8 * q);
  const ov_iv4 a = cp[0], b = cp[1];
  c8[0] = a.x; c8[1] = a.y; c8[2] = a.z; c8[3] = a.w;
  c8[4] = b.x; c8[5] = b.y; c8[6] = b.z; c8[7] = b.w;
  if constexpr (sizeof(T) == 4) {
    gmem<ov_fv4>* vp = (gmem<ov_fv4>*)gp(vals) + 2 * q;
    const ov_fv4 u = vp[0], v = vp[1];
    w8[0] = u.x; w8[1] = u.y; w8[2] = u.z; w8[3] = u.w;
    w8[4] = v.x; w8[5] = v.y; w8[6] = v.z; w8[7] = v.w;
  } else {
    gmem<ov_dv2>* vp = (gmem<ov_dv2>*)gp(vals) + 4 * q;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const ov_dv2 u = vp[k];
      w8[2 * k] = u.x;
      w8[2 * k + 1] = u.y;
    }
  }
}

template <typename T, int INTERLEAVED, int NR>
__global__ void __launch_bounds__(256) k_interp_apply(const int32_t* __restrict__ cols, const T* __restrict__ vals,
                                                     const long long* __restrict__ d_count, long long capacity,
                                                     const T* __restrict__ x, long long total, int nrhs,
                                                     T* __restrict__ y) {
  const long long n = min(*d_count, capacity);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    int c8[8];
    T w8[8];
    load_row<T>(cols, vals, q, c8, w8);
    // loads first, for every entry (an absent one reads node 0), so that all
    // of a row's gathers are in flight together; absent entries add nothing
    bool on[8];
    long long idx[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      on[c] = c8[c] >= 0;
      idx[c] = on[c] ? c8[c] : 0;
    }
    if constexpr (INTERLEAVED && NR == 4) {
      typedef typename Vec4<T>::type V;
      V v[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) v[c] = ((gmem<V>*)gp(x))[idx[c]];
      V acc = (V)0;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (on[c]) acc += w8[c] * v[c];
      ((V*)y)[q] = acc;
    } else {
      for (int r = 0; r < nrhs; ++r) {
        T v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c)
          v[c] = INTERLEAVED ? gp(x)[idx[c] * nrhs + r] : gp(x)[(long long)r * total + idx[c]];
        T acc = 0;
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (on[c]) acc += w8[c] * v[c];
        if (INTERLEAVED)
          y[q * nrhs + r] = acc;
        else
          y[(long long)r * capacity + q] = acc;
      }
    }
  }
}

template <typename T>
hipError_t launch_apply_t(ov_ctx* ctx, const int32_t* cols, const T* vals, const long long* d_count,
                          long long capacity, const T* x, int nrhs, int layout, T* y, hipStream_t st) {
  // one row per thread: a gather kernel wants every wave the chip can hold
  long long grid = (capacity + 255) / 256;
  if (grid > (1LL << 30)) grid = 1LL << 30;
  const long long total = ctx->node_off.back();
  const dim3 g((unsigned)grid), b(256);
  if (layout == 0)
    hipLaunchKernelGGL((k_interp_apply<T, 0, 0>), g, b, 0, st, cols, vals, d_count, capacity, x, total, nrhs, y);
  else if (nrhs == 4)
    hipLaunchKernelGGL((k_interp_apply<T, 1, 4>), g, b, 0, st, cols, vals, d_count, capacity, x, total, nrhs, y);
  else
    hipLaunchKernelGGL((k_interp_apply<T, 1, 0>), g, b, 0, st, cols, vals, d_count, capacity, x, total, nrhs, y);
  return hipGetLastError();
}

}  // namespace ov

using namespace ov;

static int ready(ov_ctx* ctx) {
  if (!ctx) return OV_EINVAL;
  if (!ctx->finalized) return fail(ctx, OV_ESTATE, "step call before ov_finalize");
  return OV_OK;
}

extern "C" {

int overset_frame_velocity(ov_ctx* ctx, const double* poses, const int32_t* q_grid, const int32_t* donor_grid,
                           const int64_t* d_count, int64_t capacity, void* out, void* stream) {
  int rc = ready(ctx);
  if (rc) return rc;
  if (capacity < 0) return fail(ctx, OV_EINVAL, "overset_frame_velocity: negative capacity");
  if (capacity == 0) return OV_OK;
  if (!poses || !q_grid || !donor_grid || !d_count || !out)
    return fail(ctx, OV_EINVAL, "overset_frame_velocity: null pointer");
  hipError_t e = launch_frame_velocity(ctx, poses, q_grid, donor_grid, (const long long*)d_count, capacity, out,
                                       (hipStream_t)stream);
  return e == hipSuccess ? OV_OK : hip_fail(ctx, e, "overset_frame_velocity");
}

int overset_interp_matrix(ov_ctx* ctx, const int32_t* donor_grid, const int32_t* donor_cell, const void* s,
                          const int64_t* d_count, int64_t capacity, int32_t* cols, void* vals, void* stream) {
  int rc = ready(ctx);
  if (rc) return rc;
  if (capacity < 0) return fail(ctx, OV_EINVAL, "overset_interp_matrix: negative capacity");
  if (capacity == 0) return OV_OK;
  if (!donor_grid || !donor_cell || !s || !d_count || !cols || !vals)
    return fail(ctx, OV_EINVAL, "overset_interp_matrix: null pointer");
  if (ctx->node_off.back() >= (1LL << 31))
    return fail(ctx, OV_EDIMS, "overset_interp_matrix: 32-bit column indices need fewer than 2^31 nodes");
  const long long grid = grid_size_for(ctx, capacity, 256);
  hipStream_t st = (hipStream_t)stream;
  if (ctx->precision == OV_MIXED)
    hipLaunchKernelGGL(k_interp_matrix<float>, dim3((unsigned)grid), dim3(256), 0, st, ctx->d_grids, donor_grid,
                       donor_cell, (const float*)s, (const long long*)d_count, capacity, cols, (float*)vals);
  else
    hipLaunchKernelGGL(k_interp_matrix<double>, dim3((unsigned)grid), dim3(256), 0, st, ctx->d_grids, donor_grid,
                       donor_cell, (const double*)s, (const long long*)d_count, capacity, cols, (double*)vals);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? OV_OK : hip_fail(ctx, e, "overset_interp_matrix");
}

int overset_interp_apply(ov_ctx* ctx, const int32_t* cols, const void* vals, const int64_t* d_count,
                         int64_t capacity, const void* x, int32_t nrhs, int32_t layout, void* y, void* stream) {
  int rc = ready(ctx);
  if (rc) return rc;
  if (capacity < 0 || nrhs < 0) return fail(ctx, OV_EINVAL, "overset_interp_apply: negative capacity or nrhs");
  if (layout != 0 && layout != 1) return fail(ctx, OV_EINVAL, "overset_interp_apply: layout must be 0 or 1");
  if (capacity == 0 || nrhs == 0) return OV_OK;
  if (!cols || !vals || !d_count || !x || !y) return fail(ctx, OV_EINVAL, "overset_interp_apply: null pointer");
  const size_t es = ctx->precision == OV_MIXED ? 4 : 8;
  const size_t vec = (layout == 1 && nrhs == 4) ? 4 * es : es;
  if (((uintptr_t)cols & 15) || ((uintptr_t)vals & 15) || ((uintptr_t)x % vec) || ((uintptr_t)y % vec))
    return fail(ctx, OV_EINVAL, "overset_interp_apply: cols and vals need 16-byte alignment, x and y that of "
                                "one node's values (interleaved, 4 vectors) or of one value");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (ctx->precision == OV_MIXED)
    e = launch_apply_t<float>(ctx, cols, (const float*)vals, (const long long*)d_count, capacity, (const float*)x,
                              (int)nrhs, (int)layout, (float*)y, st);
  else
    e = launch_apply_t<double>(ctx, cols, (const double*)vals, (const long long*)d_count, capacity,
                               (const double*)x, (int)nrhs, (int)layout, (double*)y, st);
  return e == hipSuccess ? OV_OK : hip_fail(ctx, e, "overset_interp_apply");
}

}  // extern "C"
