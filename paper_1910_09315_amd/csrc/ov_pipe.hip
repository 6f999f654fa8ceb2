// Native step pipelines.
//
// Consecutive steps rotate through caller-owned buffer sets and run in
// stages on separate streams:
//  two stages (ov_pipe_create): front = hole cut + fringe marking +
//    compaction, back = transform + donor search + interpolation; two sets.
//    front(t+1) overlaps back(t).
//  three stages (ov_pipe_create3): A = hole cut, B = fringe marking +
//    compaction, C = the back half; three sets. A(t+1), B(t) and C(t-1) run
//    at the same time. Set k uses front-half scratch slot k of the context
//    (near-tile list, chunk-list length, stamp), so A and B of one step share
//    a slot and no two steps in flight do.
// Events keep the order every buffer needs: B(t) after A(t); C(t) after
// B(t); A(t) after C(t - nsets), the last reader of its buffer set and slot.
// Stages of one kind follow one another on their stream, which keeps the
// warm start of the walk exact. All launches are issued here in C++.
//
// With graphs on (ov_pipe_use_graphs), each stage of each buffer set is
// captured once as a single-stream HIP graph reading its poses from a
// per-set device slot; a step is then one pose copy, one graph launch per
// stage and the events: the host cost of a step no longer grows with the
// number of kernels.
#include <hip/hip_runtime.h>

#include <vector>

#include "ov_internal.h"

struct ov_pipe {
  ov_ctx* ctx = nullptr;
  int nf = 0;
  int nsets = 2;
  ov_step_buffers sets[3];
  const void* fields = nullptr;
  hipStream_t sa = nullptr, sb = nullptr, sc = nullptr;  // sb == sa with two stages
  hipEvent_t a_done[3] = {}, b_done[3] = {}, c_done[3] = {};
  hipEvent_t join[3] = {};
  long long t = 0;
  // graphs
  bool graphs = false;
  double* poses_slot = nullptr;  // nsets x ngrids x 12
  hipGraph_t g[3][3] = {};       // [set][stage]
  hipGraphExec_t gx[3][3] = {};
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

static int slot_of(const ov_pipe* p, int k) { return p->nsets == 3 ? k : 0; }

// The launches of stage `stage` (0 = A, 1 = B, 2 = C) for buffer set k on
// stream s, reading poses from `poses`.
static hipError_t stage_launch(ov_pipe* p, int k, int stage, const double* poses, hipStream_t s) {
  ov_ctx* ctx = p->ctx;
  const ov_step_buffers& b = p->sets[k];
  const int slot = slot_of(p, k);
  hipError_t e = hipSuccess;
  if (stage == 0) {
    e = launch_holecut(ctx, poses, b.flags, s, slot);
  } else if (stage == 1) {
    e = launch_fringe(ctx, p->nf, b.flags, s, slot);
    if (e == hipSuccess)
      e = launch_compact(ctx, b.flags, b.q_grid, b.q_node, b.capacity, (long long*)b.d_count, s, slot);
  } else if (b.capacity > 0) {
    e = launch_transform(ctx, poses, b.q_grid, b.q_node, (const long long*)b.d_count, b.capacity, b.qx, s);
    if (e == hipSuccess)
      e = launch_donor_search(ctx, poses, b.flags, b.q_grid, b.q_node, b.qx, (const long long*)b.d_count,
                              b.capacity, b.donor_grid, b.donor_cell, b.s, b.status, s);
    if (e == hipSuccess && p->fields)
      e = launch_interp(ctx, b.donor_grid, b.donor_cell, b.s, (const long long*)b.d_count, b.capacity, p->fields,
                        b.out, s);
  }
  return e;
}

static void destroy_graphs(ov_pipe* p) {
  for (int k = 0; k < 3; ++k)
    for (int st = 0; st < 3; ++st) {
      if (p->gx[k][st]) (void)hipGraphExecDestroy(p->gx[k][st]);
      if (p->g[k][st]) (void)hipGraphDestroy(p->g[k][st]);
      p->gx[k][st] = nullptr;
      p->g[k][st] = nullptr;
    }
  if (p->poses_slot) (void)hipFree(p->poses_slot);
  p->poses_slot = nullptr;
  p->graphs = false;
}

static int pipe_create(ov_ctx* ctx, int32_t nf, int nsets, const ov_step_buffers* sets, const void* fields,
                       hipStream_t sa, hipStream_t sb, hipStream_t sc, int32_t max_timed, ov_pipe** out) {
  if (!ctx || !sets || !out) return OV_EINVAL;
  *out = nullptr;
  if (!ctx->finalized) return fail(ctx, OV_ESTATE, "ov_pipe_create before ov_finalize");
  if (nf < 0 || nf > kMaxNf) return fail(ctx, OV_EINVAL, "ov_pipe_create: nf must be in 0..%d", kMaxNf);
  if (sa == sc || sb == sc || (nsets == 3 && sa == sb))
    return fail(ctx, OV_EINVAL, "ov_pipe_create: the streams must differ");
  if (max_timed < 0) return fail(ctx, OV_EINVAL, "ov_pipe_create: negative max_timed");
  for (int k = 0; k < nsets; ++k) {
    const ov_step_buffers& b = sets[k];
    if (!b.flags || !b.d_count || b.capacity < 0 || (b.capacity > 0 && (!b.q_grid || !b.q_node || !b.qx ||
                                                                        !b.donor_grid || !b.donor_cell || !b.s ||
                                                                        !b.status || (fields && !b.out))))
      return fail(ctx, OV_EINVAL, "ov_pipe_create: incomplete buffer set");
    if (((uintptr_t)b.flags & 15) != 0) return fail(ctx, OV_EINVAL, "ov_pipe_create: flags must be 16-byte aligned");
  }
  ov_pipe* p = new ov_pipe();
  p->ctx = ctx;
  p->nf = nf;
  p->nsets = nsets;
  for (int k = 0; k < nsets; ++k) p->sets[k] = sets[k];
  p->fields = fields;
  p->sa = sa;
  p->sb = sb;
  p->sc = sc;
  bool ok = true;
  for (int k = 0; k < 3 && ok; ++k) {
    ok &= hipEventCreateWithFlags(&p->a_done[k], hipEventDisableTiming) == hipSuccess;
    ok &= hipEventCreateWithFlags(&p->b_done[k], hipEventDisableTiming) == hipSuccess;
    ok &= hipEventCreateWithFlags(&p->c_done[k], hipEventDisableTiming) == hipSuccess;
    ok &= hipEventCreateWithFlags(&p->join[k], hipEventDisableTiming) == hipSuccess;
  }
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

extern "C" {

int ov_pipe_create(ov_ctx* ctx, int32_t nf, const ov_step_buffers* sets, const void* fields, void* stream_front,
                   void* stream_back, int32_t max_timed, ov_pipe** out) {
  return pipe_create(ctx, nf, 2, sets, fields, (hipStream_t)stream_front, (hipStream_t)stream_front,
                     (hipStream_t)stream_back, max_timed, out);
}

int ov_pipe_create3(ov_ctx* ctx, int32_t nf, const ov_step_buffers* sets, const void* fields, void* stream_a,
                    void* stream_b, void* stream_c, int32_t max_timed, ov_pipe** out) {
  return pipe_create(ctx, nf, 3, sets, fields, (hipStream_t)stream_a, (hipStream_t)stream_b, (hipStream_t)stream_c,
                     max_timed, out);
}

int ov_pipe_use_graphs(ov_pipe* p, int32_t on) {
  if (!p) return OV_EINVAL;
  if (p->t != 0) return pipe_fail(p, OV_ESTATE, "ov_pipe_use_graphs after the first submit");
  destroy_graphs(p);
  if (!on) return OV_OK;
  ov_ctx* ctx = p->ctx;
  const size_t per_set = 12 * ctx->grids.size();
  hipStream_t cap = nullptr;
  hipError_t e = hipMalloc(&p->poses_slot, sizeof(double) * per_set * p->nsets);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  const bool three = p->nsets == 3;
  for (int k = 0; k < p->nsets && e == hipSuccess; ++k) {
    const double* poses = p->poses_slot + per_set * k;
    for (int g = 0; g < (three ? 3 : 2) && e == hipSuccess; ++g) {
      // with two stages, graph 0 holds the whole front (A then B) and graph 1 the back
      e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      hipError_t le = hipSuccess;
      if (e == hipSuccess) {
        if (three) {
          le = stage_launch(p, k, g, poses, cap);
        } else if (g == 0) {
          le = stage_launch(p, k, 0, poses, cap);
          if (le == hipSuccess) le = stage_launch(p, k, 1, poses, cap);
        } else {
          le = stage_launch(p, k, 2, poses, cap);
        }
      }
      hipGraph_t graph = nullptr;
      if (e == hipSuccess) e = hipStreamEndCapture(cap, &graph);
      p->g[k][g] = graph;
      if (e == hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&p->gx[k][g], graph, nullptr, nullptr, 0);
    }
  }
  if (cap) (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    destroy_graphs(p);
    return hip_fail(ctx, e, "ov_pipe_use_graphs");
  }
  p->graphs = true;
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
  const long long t = p->t;
  const int k = (int)(t % p->nsets);
  const ov_step_buffers& b = p->sets[k];
  const bool three = p->nsets == 3;
  hipError_t e = hipSuccess;
  // A: hole cut (with two stages: the whole front half), after the last
  // reader of this buffer set and slot
  if (t >= p->nsets) e = hipStreamWaitEvent(p->sa, p->c_done[k], 0);
  const double* ps = poses;
  if (e == hipSuccess && p->graphs) {
    double* slot = p->poses_slot + 12 * ctx->grids.size() * k;
    e = hipMemcpyAsync(slot, poses, sizeof(double) * 12 * ctx->grids.size(), hipMemcpyDeviceToDevice, p->sa);
    ps = slot;
  }
  const bool timed = p->timing && p->ntimed < (int)p->tb.size();
  if (e == hipSuccess && timed) e = hipEventRecord(p->tb[p->ntimed], p->sa);
  if (e == hipSuccess) e = p->graphs ? hipGraphLaunch(p->gx[k][0], p->sa) : stage_launch(p, k, 0, ps, p->sa);
  if (e == hipSuccess && timed) e = hipEventRecord(p->te[p->ntimed], p->sa);
  if (three) {
    if (e == hipSuccess) e = hipEventRecord(p->a_done[k], p->sa);
    // B: fringe marking and compaction
    if (e == hipSuccess) e = hipStreamWaitEvent(p->sb, p->a_done[k], 0);
    if (e == hipSuccess) e = p->graphs ? hipGraphLaunch(p->gx[k][1], p->sb) : stage_launch(p, k, 1, ps, p->sb);
  } else if (e == hipSuccess && !p->graphs) {
    e = stage_launch(p, k, 1, ps, p->sa);  // the front half continues on its stream
  }
  if (e == hipSuccess) e = hipEventRecord(p->b_done[k], p->sb);
  // C: transform, donor search, interpolation
  if (e == hipSuccess) e = hipStreamWaitEvent(p->sc, p->b_done[k], 0);
  if (e == hipSuccess)
    e = p->graphs ? hipGraphLaunch(p->gx[k][three ? 2 : 1], p->sc) : stage_launch(p, k, 2, ps, p->sc);
  if (e == hipSuccess && count_out) {
    hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, p->sc, (long long*)count_out,
                       (const long long*)b.d_count);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(p->c_done[k], p->sc);
  if (e != hipSuccess) return hip_fail(ctx, e, "ov_pipe_submit");
  if (timed) ++p->ntimed;
  ++p->t;
  return OV_OK;
}

int ov_pipe_submit_many(ov_pipe* p, const double* poses, int64_t pose_stride, int64_t n, int64_t* counts_out) {
  if (!p || !poses || n < 0 || pose_stride < 12 * (int64_t)p->ctx->grids.size())
    return pipe_fail(p, OV_EINVAL, "ov_pipe_submit_many: bad argument");
  for (int64_t i = 0; i < n; ++i) {
    int rc = ov_pipe_submit(p, poses + pose_stride * i, counts_out ? counts_out + i : nullptr);
    if (rc != OV_OK) return rc;
  }
  return OV_OK;
}

int ov_pipe_join(ov_pipe* p, void* stream) {
  if (!p) return OV_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipStream_t st[3] = {p->sa, p->sb, p->sc};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 3 && e == hipSuccess; ++i) {
    e = hipEventRecord(p->join[i], st[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join[i], 0);
  }
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
  hipStream_t st[3] = {p->sa, p->sb, p->sc};
  for (auto q : st)
    if (q) (void)hipStreamSynchronize(q);
  destroy_graphs(p);
  for (int k = 0; k < 3; ++k) {
    if (p->a_done[k]) (void)hipEventDestroy(p->a_done[k]);
    if (p->b_done[k]) (void)hipEventDestroy(p->b_done[k]);
    if (p->c_done[k]) (void)hipEventDestroy(p->c_done[k]);
    if (p->join[k]) (void)hipEventDestroy(p->join[k]);
  }
  for (auto ev : p->tb)
    if (ev) (void)hipEventDestroy(ev);
  for (auto ev : p->te)
    if (ev) (void)hipEventDestroy(ev);
  delete p;
  return OV_OK;
}

}  // extern "C"
