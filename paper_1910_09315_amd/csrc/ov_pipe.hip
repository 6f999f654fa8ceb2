// Native two-stream step pipeline.
//
// Consecutive steps alternate between two caller-owned buffer sets. The
// front half of a step (hole cut, fringe marking and compaction) runs on one
// stream, the back half (transform, donor search, interpolation) on another:
// the front half of step t+1 overlaps the back half of step t. Events keep
// the order every buffer needs: back(t) after front(t); front(t+2) after
// back(t), which last read set t%2; back(t+1) after back(t) by stream order,
// which keeps the warm start of the walk exact. The library's scratch is
// split the same way (the front half only touches front-half scratch), so no
// other ordering is needed. All launches are issued here in C++, so a step
// costs the host one call.
#include <hip/hip_runtime.h>

#include <vector>

#include "ov_internal.h"

struct ov_pipe {
  ov_ctx* ctx = nullptr;
  int nf = 0;
  ov_step_buffers sets[2];
  const void* fields = nullptr;
  hipStream_t front = nullptr, back = nullptr;
  hipEvent_t front_done[2] = {nullptr, nullptr}, back_done[2] = {nullptr, nullptr};
  hipEvent_t join_front = nullptr, join_back = nullptr;
  bool started[2] = {false, false};
  long long t = 0;
  // hole-cut timing (optional)
  std::vector<hipEvent_t> tb, te;
  int ntimed = 0;
  bool timing = false;
};

namespace ov {

__global__ void k_copy_count(long long* __restrict__ dst, const long long* __restrict__ src) { *dst = *src; }

}  // namespace ov

using namespace ov;

static int pipe_fail(ov_pipe* p, int code, const char* msg) { return fail(p ? p->ctx : nullptr, code, "%s", msg); }

extern "C" {

int ov_pipe_create(ov_ctx* ctx, int32_t nf, const ov_step_buffers* sets, const void* fields, void* stream_front,
                   void* stream_back, int32_t max_timed, ov_pipe** out) {
  if (!ctx || !sets || !out) return OV_EINVAL;
  *out = nullptr;
  if (!ctx->finalized) return fail(ctx, OV_ESTATE, "ov_pipe_create before ov_finalize");
  if (nf < 0 || nf > kMaxNf) return fail(ctx, OV_EINVAL, "ov_pipe_create: nf must be in 0..%d", kMaxNf);
  if (stream_front == stream_back) return fail(ctx, OV_EINVAL, "ov_pipe_create: the two streams must differ");
  if (max_timed < 0) return fail(ctx, OV_EINVAL, "ov_pipe_create: negative max_timed");
  for (int k = 0; k < 2; ++k) {
    const ov_step_buffers& b = sets[k];
    if (!b.flags || !b.d_count || b.capacity < 0 || (b.capacity > 0 && (!b.q_grid || !b.q_node || !b.qx ||
                                                                        !b.donor_grid || !b.donor_cell || !b.s ||
                                                                        !b.status || (fields && !b.out))))
      return fail(ctx, OV_EINVAL, "ov_pipe_create: incomplete buffer set %d", k);
    if (((uintptr_t)b.flags & 15) != 0) return fail(ctx, OV_EINVAL, "ov_pipe_create: flags must be 16-byte aligned");
  }
  ov_pipe* p = new ov_pipe();
  p->ctx = ctx;
  p->nf = nf;
  p->sets[0] = sets[0];
  p->sets[1] = sets[1];
  p->fields = fields;
  p->front = (hipStream_t)stream_front;
  p->back = (hipStream_t)stream_back;
  bool ok = true;
  for (int k = 0; k < 2 && ok; ++k) {
    ok &= hipEventCreateWithFlags(&p->front_done[k], hipEventDisableTiming) == hipSuccess;
    ok &= hipEventCreateWithFlags(&p->back_done[k], hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipEventCreateWithFlags(&p->join_front, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&p->join_back, hipEventDisableTiming) == hipSuccess;
  p->tb.assign(max_timed, nullptr);
  p->te.assign(max_timed, nullptr);
  for (int i = 0; i < max_timed && ok; ++i) {
    ok &= hipEventCreate(&p->tb[i]) == hipSuccess;
    ok &= hipEventCreate(&p->te[i]) == hipSuccess;
  }
  if (!ok) {
    ov_pipe_destroy(p);
    return fail(ctx, OV_EHIP, "ov_pipe_create: event creation failed");
  }
  *out = p;
  return OV_OK;
}

int ov_pipe_set_timing(ov_pipe* p, int32_t on) {
  if (!p) return OV_EINVAL;
  p->timing = on != 0;
  return OV_OK;
}

int ov_pipe_submit(ov_pipe* p, const double* poses, int64_t* count_out) {
  if (!p || !poses) return pipe_fail(p, OV_EINVAL, "ov_pipe_submit: null argument");
  ov_ctx* ctx = p->ctx;
  const int k = (int)(p->t & 1);
  const ov_step_buffers& b = p->sets[k];
  hipError_t e = hipSuccess;
  // front half
  if (p->started[k]) e = hipStreamWaitEvent(p->front, p->back_done[k], 0);
  const bool timed = p->timing && p->ntimed < (int)p->tb.size();
  if (e == hipSuccess && timed) e = hipEventRecord(p->tb[p->ntimed], p->front);
  if (e == hipSuccess) e = launch_holecut(ctx, poses, b.flags, p->front);
  if (e == hipSuccess && timed) e = hipEventRecord(p->te[p->ntimed], p->front);
  if (e == hipSuccess) e = launch_fringe(ctx, p->nf, b.flags, p->front);
  if (e == hipSuccess)
    e = launch_compact(ctx, b.flags, b.q_grid, b.q_node, b.capacity, (long long*)b.d_count, p->front);
  if (e == hipSuccess) e = hipEventRecord(p->front_done[k], p->front);
  // back half
  if (e == hipSuccess) e = hipStreamWaitEvent(p->back, p->front_done[k], 0);
  if (e == hipSuccess && b.capacity > 0) {
    e = launch_transform(ctx, poses, b.q_grid, b.q_node, (const long long*)b.d_count, b.capacity, b.qx, p->back);
    if (e == hipSuccess)
      e = launch_donor_search(ctx, poses, b.flags, b.q_grid, b.q_node, b.qx, (const long long*)b.d_count,
                              b.capacity, b.donor_grid, b.donor_cell, b.s, b.status, p->back);
    if (e == hipSuccess && p->fields)
      e = launch_interp(ctx, b.donor_grid, b.donor_cell, b.s, (const long long*)b.d_count, b.capacity, p->fields,
                        b.out, p->back);
  }
  if (e == hipSuccess && count_out) {
    hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, p->back, (long long*)count_out,
                       (const long long*)b.d_count);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(p->back_done[k], p->back);
  if (e != hipSuccess) return hip_fail(ctx, e, "ov_pipe_submit");
  if (timed) ++p->ntimed;
  p->started[k] = true;
  ++p->t;
  return OV_OK;
}

int ov_pipe_join(ov_pipe* p, void* stream) {
  if (!p) return OV_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipEventRecord(p->join_front, p->front);
  if (e == hipSuccess) e = hipEventRecord(p->join_back, p->back);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join_front, 0);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join_back, 0);
  return e == hipSuccess ? OV_OK : hip_fail(p->ctx, e, "ov_pipe_join");
}

int ov_pipe_holecut_times(ov_pipe* p, float* ms_out, int32_t max, int32_t* n_out) {
  if (!p || !n_out || (max > 0 && !ms_out)) return OV_EINVAL;
  int n = p->ntimed < max ? p->ntimed : max;
  for (int i = 0; i < n; ++i) {
    hipError_t e = hipEventSynchronize(p->te[i]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_out[i], p->tb[i], p->te[i]);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "ov_pipe_holecut_times");
  }
  *n_out = n;
  p->ntimed = 0;
  return OV_OK;
}

int ov_pipe_destroy(ov_pipe* p) {
  if (!p) return OV_EINVAL;
  if (p->front) (void)hipStreamSynchronize(p->front);
  if (p->back) (void)hipStreamSynchronize(p->back);
  for (int k = 0; k < 2; ++k) {
    if (p->front_done[k]) (void)hipEventDestroy(p->front_done[k]);
    if (p->back_done[k]) (void)hipEventDestroy(p->back_done[k]);
  }
  if (p->join_front) (void)hipEventDestroy(p->join_front);
  if (p->join_back) (void)hipEventDestroy(p->join_back);
  for (auto ev : p->tb)
    if (ev) (void)hipEventDestroy(ev);
  for (auto ev : p->te)
    if (ev) (void)hipEventDestroy(ev);
  delete p;
  return OV_OK;
}

}  // extern "C"
