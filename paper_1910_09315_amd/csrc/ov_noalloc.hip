// The fringe call without allocation, for callers that cannot allocate
// device memory (work under HIP graph capture, tight serving loops,
// harnesses that forbid it).
//
// overset_fringe_compact_noalloc runs the kernels of overset_fringe_compact
// (near list from the flags, fringe marking, count / scan / write
// compaction) with their per-call scratch (near-tile list and marks, chunk
// list and marks, per-chunk and per-superchunk counts, superchunk offsets)
// in one file-scope device array, `scratch`, instead of the context's
// memory. The array has a fixed size; a problem whose scratch does not fit
// is refused before any launch. Every call on a device shares that device's
// copy of the array: each call first clears what must start at zero, and
// calls that overlap on one device (streams not ordered against each
// other) race on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "ov_internal.h"

namespace ov {

constexpr size_t kStaticScratchBytes = size_t(6) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_looked_up[kMaxDevices] = {};
void* g_addr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
}  // namespace

// The device address of this device's copy of `scratch`, looked up once per
// device; the caller has made `device` current. In host code the array's
// name is only a stand-in: kernels and copies must get this address.
hipError_t static_scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_looked_up[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_err[device] = e;
    g_addr[device] = e == hipSuccess ? p : nullptr;
    g_looked_up[device] = true;
  }
  *out = g_addr[device];
  return g_err[device];
}

// Carves the fringe pass's scratch for ctx out of the array at `base`;
// returns the bytes needed (larger than kStaticScratchBytes: does not fit).
static size_t static_layout(const ov_ctx* ctx, unsigned char* base, FrontScratch& fs) {
  const long long nt = std::max(1LL, ctx->total_tiles);
  const long long nch = std::max(1LL, ctx->nchunks);
  const long long nsc = kSuperSlots * std::max(1LL, ctx->nsuper);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off = align256(off + bytes);
    return p;
  };
  unsigned int* hdr = reinterpret_cast<unsigned int*>(take(4 * sizeof(unsigned int)));
  fs.counter = hdr;
  fs.stamp = hdr + 1;
  fs.near_count = reinterpret_cast<int32_t*>(hdr + 2);
  fs.chunk_list_count = reinterpret_cast<int32_t*>(hdr + 3);
  fs.super_counts = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nsc));
  fs.super_offsets = reinterpret_cast<long long*>(take(sizeof(long long) * (std::max(1LL, ctx->nsuper) + 1)));
  fs.chunk_counts = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * nch));
  fs.chunk_stamp = reinterpret_cast<unsigned int*>(take(sizeof(unsigned int) * nch));
  fs.chunk_list = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nch));
  fs.tile_near = reinterpret_cast<unsigned int*>(take(sizeof(unsigned int) * nt));
  fs.near_list = reinterpret_cast<int4*>(take(sizeof(int4) * nt));
  return off;
}

// Starts a call on the static scratch: clears the marks and counts the
// kernels test against the stamp or add to, sets the stamp to 1 (0 means
// "never listed"), empties the lists and puts the context's static chunks
// (those holding outer-boundary nodes) at the head of the chunk list.
__global__ void __launch_bounds__(256) k_static_begin(FrontScratch fs, long long nt, long long nchunks,
                                                     long long nsc, const int32_t* __restrict__ static_list,
                                                     long long n_static) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) {
    *fs.counter = 1u;
    *fs.stamp = 1u;
    *fs.near_count = 0;
    *fs.chunk_list_count = 0;
  }
  for (long long i = i0; i < nt; i += stride) fs.tile_near[i] = 0u;
  for (long long i = i0; i < nchunks; i += stride) {
    fs.chunk_stamp[i] = 0u;
    fs.chunk_counts[i] = 0ull;
  }
  for (long long i = i0; i < nsc; i += stride) fs.super_counts[i] = 0;
  for (long long i = i0; i < n_static; i += stride) fs.chunk_list[i] = static_list[i];
}

}  // namespace ov

using namespace ov;

extern "C" int overset_fringe_compact_noalloc(ov_ctx* ctx, int32_t nf, uint8_t* flags, int32_t* q_grid,
                                              int32_t* q_node, int64_t capacity, int64_t* d_count, void* stream) {
  if (!ctx) return OV_EINVAL;
  if (!ctx->finalized) return fail(ctx, OV_ESTATE, "step call before ov_finalize");
  if (!flags || !d_count || (capacity > 0 && (!q_grid || !q_node)))
    return fail(ctx, OV_EINVAL, "overset_fringe_compact_noalloc: null pointer");
  if (((uintptr_t)flags & 15) != 0)
    return fail(ctx, OV_EINVAL, "overset_fringe_compact_noalloc: flags must be 16-byte aligned");
  if (nf < 0 || nf > kMaxNf)
    return fail(ctx, OV_EINVAL, "overset_fringe_compact_noalloc: nf must be in 0..%d", kMaxNf);
  if (capacity < 0) return fail(ctx, OV_EINVAL, "overset_fringe_compact_noalloc: negative capacity");
  if (!ctx->static_scratch)
    return fail(ctx, OV_EHIP, "overset_fringe_compact_noalloc: the static scratch array has no device address");
  FrontScratch fs;
  const size_t need = static_layout(ctx, static_cast<unsigned char*>(ctx->static_scratch), fs);
  if (need > kStaticScratchBytes)
    return fail(ctx, OV_ECAPACITY,
                "overset_fringe_compact_noalloc: %lld tiles and %lld chunks need %zu bytes of scratch, more than "
                "the static %zu",
                ctx->total_tiles, ctx->nchunks, need, kStaticScratchBytes);
  hipStream_t s = (hipStream_t)stream;
  const long long nt = std::max(1LL, ctx->total_tiles), nch = std::max(1LL, ctx->nchunks);
  const long long nsc = kSuperSlots * std::max(1LL, ctx->nsuper);
  const long long items = std::max(std::max(nt, nch), std::max(nsc, ctx->n_static_chunks));
  const long long blocks = std::max(1LL, std::min((items + 255) / 256, (long long)ctx->num_cus * 4));
  hipLaunchKernelGGL(k_static_begin, dim3((unsigned)blocks), dim3(256), 0, s, fs, nt, nch, nsc,
                     (const int32_t*)ctx->d_chunk_list, ctx->n_static_chunks);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_near_list_in(ctx, flags, s, fs);
  if (e == hipSuccess) e = launch_fringe_in(ctx, nf, flags, s, fs);
  if (e == hipSuccess) e = launch_compact_in(ctx, flags, q_grid, q_node, capacity, (long long*)d_count, s, fs, false);
  return e == hipSuccess ? OV_OK : hip_fail(ctx, e, "overset_fringe_compact_noalloc");
}
