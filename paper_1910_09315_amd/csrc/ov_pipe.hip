// Native step executors.
//
// A step is three stages: A = hole cut, B = fringe marking + compaction,
// C = the back half (transform, donor search, interpolation). Consecutive
// steps rotate through caller-owned buffer sets; the stages run on one,
// two or three streams:
//  one stream (ov_pipe_create1): A, B, C in stream order, one buffer set,
//    no events. The cheapest for the host: a step is its kernel launches.
//  two streams (ov_pipe_create): A and B on the front stream, C on the back
//    stream; two sets. front(t+1) overlaps C(t).
//  three streams (ov_pipe_create3): A, B and C each on its own stream; three
//    sets. A(t+1), B(t) and C(t-1) run at the same time.
// Set k uses front-half scratch slot k of the context (near-tile list,
// chunk-list length, stamp), so A and B of one step share a slot and no two
// steps in flight do. The order every buffer needs: a stage runs after the
// previous stage of its step, and the first stage of step t after
// the last stage of step t - nsets, the last reader of its buffer set and
// slot. Stages of one kind follow one another on their stream, which keeps
// the warm start of the walk exact. The order between streams is kept with
// stream memory operations on 64-bit sequence counters in device memory:
// after group g of step t its stream writes t + 1 to counter g, and a
// stream that must follow it waits until the counter is >= t + 1 (the
// counters only grow). These cost the host far less than event records and
// event waits; still, the stream count is a trade between host time and
// overlap on the device.
//
// With graphs on (ov_pipe_use_graphs), the stages each stream runs for each
// buffer set are captured once as a single-stream HIP graph reading its
// poses from a per-set device slot; a step is then one pose copy, one graph
// launch per stream and the counter operations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "ov_internal.h"

struct ov_pipe {
  ov_ctx* ctx = nullptr;
  int nf = 0;
  int nsets = 2;  // = number of streams
  ov_step_buffers sets[3];
  const void* fields = nullptr;
  hipStream_t st[3] = {};          // stream of each group of stages
  unsigned long long* seq = nullptr;  // device: [group] = 1 + the last step whose group is done
  hipEvent_t join[3] = {};
  long long t = 0;
  // graphs
  bool graphs = false;
  double* poses_slot = nullptr;  // nsets x ngrids x 12
  hipGraphExec_t gx[3][3] = {};  // [set][group]
  hipGraph_t g[3][3] = {};
  // stage timing (optional)
  std::vector<hipEvent_t> tb, te;
  int ntimed = 0;
  int timing = 0;       // time stage timed_stage of every timing-th submitted step (0: none)
  long long timing_t0 = 0;  // the first step timed: the next step submitted after the timing call
  int timed_stage = 0;  // 0 = A (hole cut), 1 = B, 2 = C
  bool timed_alone = true;  // a timed stage runs alone (extra waits) or keeps its place in the pipeline
  // the timed group runs alone: the next step's first group waits for it
  int after_group = -1;
  long long after_value = 0;
  // per buffer set: steps started on it, and the near list its current step uses
  long long uses[3] = {0, 0, 0};
  int gen[3] = {0, 0, 0};
  // deferral queue of the two-kernel back half (OV_OPT_BACK_FUSED = 2):
  // entries for the largest capacity, two step counters, then the two heads
  // of the back half's work queue (OV_OPT_BACK_QUEUE), all zeroed here
  int32_t* defer_items = nullptr;
  unsigned int* defer_count = nullptr;
  // submit_many from one host thread per stream (ov_pipe_set_threads)
  bool threads = false;
  // by-step order (ov_pipe_set_by_step): step t runs its three stages on
  // stream t mod nsets; a stage timed alone hands the next step this event
  bool by_step = false;
  hipEvent_t alone_done = nullptr;
  bool alone_pending = false;
};

using namespace ov;

static int pipe_fail(ov_pipe* p, int code, const char* msg) { return fail(p ? p->ctx : nullptr, code, "%s", msg); }

// Stream groups: group g runs stages [first_stage(g), first_stage(g + 1)).
static int first_stage(const ov_pipe* p, int g) {
  static const int one[2] = {0, 3}, two[3] = {0, 2, 3}, three[4] = {0, 1, 2, 3};
  return p->nsets == 1 ? one[g] : p->nsets == 2 ? two[g] : three[g];
}

// Launches stage `stage` (0 = A, 1 = B, 2 = C) for buffer set k on stream s,
// reading poses from `poses`; count_out (nullable) gets the query count.
// gen: the slot's near list this step writes (A) and reads (B); reset: A
// starts from the set's previous step (k_flag_reset) instead of a full fill;
// stamp: the hole cut's stamp numbered on the host, or 0 (on the device).
static hipError_t stage_launch(ov_pipe* p, int k, int stage, const double* poses, hipStream_t s,
                               long long* count_out, int gen, bool reset, unsigned int stamp = 0u) {
  ov_ctx* ctx = p->ctx;
  const ov_step_buffers& b = p->sets[k];
  const int slot = k;
  if (stage == 0) return launch_holecut(ctx, poses, b.flags, s, slot, gen, reset, stamp);
  if (stage == 1) {
    hipError_t e = launch_fringe(ctx, p->nf, b.flags, s, slot, gen);
    if (e == hipSuccess)
      e = launch_compact(ctx, b.flags, b.q_grid, b.q_node, b.capacity, (long long*)b.d_count, s, slot, true);
    return e;
  }
  return launch_back(ctx, poses, b.flags, b.q_grid, b.q_node, b.qx, (const long long*)b.d_count, b.capacity,
                     b.donor_grid, b.donor_cell, b.s, b.status, p->fields, p->fields ? b.out : nullptr, count_out,
                     s, slot, p->defer_items, p->defer_count);
}

// Also forgets the buffer sets' history, so that the next direct step of
// each set starts from a full flag fill (captured launches, or a capture
// that failed half way, leave that history undefined).
static void destroy_graphs(ov_pipe* p) {
  for (int k = 0; k < 3; ++k) {
    p->uses[k] = 0;
    p->gen[k] = 0;
  }
  for (int k = 0; k < 3; ++k)
    for (int g = 0; g < 3; ++g) {
      if (p->gx[k][g]) (void)hipGraphExecDestroy(p->gx[k][g]);
      if (p->g[k][g]) (void)hipGraphDestroy(p->g[k][g]);
      p->gx[k][g] = nullptr;
      p->g[k][g] = nullptr;
    }
  if (p->poses_slot) (void)hipFree(p->poses_slot);
  p->poses_slot = nullptr;
  p->graphs = false;
}

static int pipe_create(ov_ctx* ctx, int32_t nf, int nsets, const ov_step_buffers* sets, const void* fields,
                       const hipStream_t* streams, int32_t max_timed, ov_pipe** out) {
  if (!ctx || !sets || !out) return OV_EINVAL;
  *out = nullptr;
  if (!ctx->finalized) return fail(ctx, OV_ESTATE, "ov_pipe_create before ov_finalize");
  if (nf < 0 || nf > kMaxNf) return fail(ctx, OV_EINVAL, "ov_pipe_create: nf must be in 0..%d", kMaxNf);
  for (int a = 0; a < nsets; ++a)
    for (int b = a + 1; b < nsets; ++b)
      if (streams[a] == streams[b]) return fail(ctx, OV_EINVAL, "ov_pipe_create: the streams must differ");
  if (max_timed < 0) return fail(ctx, OV_EINVAL, "ov_pipe_create: negative max_timed");
  static_assert(kSlots >= 3, "one front-half scratch slot per buffer set");
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
  for (int k = 0; k < nsets; ++k) {
    p->sets[k] = sets[k];
    p->st[k] = streams[k];
  }
  p->fields = fields;
  bool ok = true;
  for (int g = 0; g < nsets && ok; ++g)
    ok &= hipEventCreateWithFlags(&p->join[g], hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&p->alone_done, hipEventDisableTiming) == hipSuccess;
  if (ok && nsets > 1) {
    int can = 0;
    ok = hipDeviceGetAttribute(&can, hipDeviceAttributeCanUseStreamWaitValue, ctx->device) == hipSuccess && can;
    ok = ok && hipMalloc(&p->seq, sizeof(unsigned long long) * 3) == hipSuccess;
    ok = ok && hipMemset(p->seq, 0, sizeof(unsigned long long) * 3) == hipSuccess;
  }
  long long max_cap = 1;
  for (int k = 0; k < nsets; ++k) max_cap = std::max(max_cap, (long long)sets[k].capacity);
  ok = ok && hipMalloc(&p->defer_items, sizeof(int32_t) * max_cap) == hipSuccess;
  ok = ok && hipMalloc(&p->defer_count, sizeof(unsigned int) * 4) == hipSuccess;
  ok = ok && hipMemset(p->defer_count, 0, sizeof(unsigned int) * 4) == hipSuccess;
  p->tb.assign(max_timed, nullptr);
  p->te.assign(max_timed, nullptr);
  for (int i = 0; i < max_timed && ok; ++i) {
    ok &= hipEventCreate(&p->tb[i]) == hipSuccess;
    ok &= hipEventCreate(&p->te[i]) == hipSuccess;
  }
  if (!ok) {
    ov_pipe_destroy(p);
    return fail(ctx, OV_EHIP, "ov_pipe_create: events or sequence counters could not be created");
  }
  *out = p;
  return OV_OK;
}

extern "C" {

int ov_pipe_create1(ov_ctx* ctx, int32_t nf, const ov_step_buffers* set, const void* fields, void* stream,
                    int32_t max_timed, ov_pipe** out) {
  hipStream_t s[1] = {(hipStream_t)stream};
  return pipe_create(ctx, nf, 1, set, fields, s, max_timed, out);
}

int ov_pipe_create(ov_ctx* ctx, int32_t nf, const ov_step_buffers* sets, const void* fields, void* stream_front,
                   void* stream_back, int32_t max_timed, ov_pipe** out) {
  hipStream_t s[2] = {(hipStream_t)stream_front, (hipStream_t)stream_back};
  return pipe_create(ctx, nf, 2, sets, fields, s, max_timed, out);
}

int ov_pipe_create3(ov_ctx* ctx, int32_t nf, const ov_step_buffers* sets, const void* fields, void* stream_a,
                    void* stream_b, void* stream_c, int32_t max_timed, ov_pipe** out) {
  hipStream_t s[3] = {(hipStream_t)stream_a, (hipStream_t)stream_b, (hipStream_t)stream_c};
  return pipe_create(ctx, nf, 3, sets, fields, s, max_timed, out);
}

int ov_pipe_use_graphs(ov_pipe* p, int32_t on) {
  if (!p) return OV_EINVAL;
  if (p->t != 0) return pipe_fail(p, OV_ESTATE, "ov_pipe_use_graphs after the first submit");
  if (on && p->by_step) return pipe_fail(p, OV_ESTATE, "ov_pipe_use_graphs: not with the by-step order");
  destroy_graphs(p);  // (the next direct step of every set starts from a full fill)
  if (!on) return OV_OK;
  p->graphs = true;  // (captured steps write every flag and use near list 0)
  ov_ctx* ctx = p->ctx;
  const size_t per_set = 12 * ctx->grids.size();
  hipStream_t cap = nullptr;
  hipError_t e = hipMalloc(&p->poses_slot, sizeof(double) * per_set * p->nsets);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  for (int k = 0; k < p->nsets && e == hipSuccess; ++k) {
    const double* poses = p->poses_slot + per_set * k;
    for (int g = 0; g < p->nsets && e == hipSuccess; ++g) {
      e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      hipError_t le = hipSuccess;
      for (int stage = first_stage(p, g); stage < first_stage(p, g + 1) && e == hipSuccess && le == hipSuccess;
           ++stage)
        le = stage_launch(p, k, stage, poses, cap, nullptr, 0, false);  // (captured steps: full fill, list 0)
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

int ov_pipe_set_timing_mode(ov_pipe* p, int32_t every, int32_t stage, int32_t alone) {
  if (!p) return OV_EINVAL;
  if (every < 0 || stage < 0 || stage > 2 || alone < 0 || alone > 1)
    return pipe_fail(p, OV_EINVAL, "ov_pipe_set_timing: bad argument");
  p->timing = every;
  p->timing_t0 = p->t;
  p->timed_stage = stage;
  p->timed_alone = alone != 0;
  return OV_OK;
}

int ov_pipe_set_timing(ov_pipe* p, int32_t every, int32_t stage) { return ov_pipe_set_timing_mode(p, every, stage, 1); }

// One step in the by-step order: all three stages on stream t mod nsets (in
// stream order after the step that used this buffer set before). Only the
// back half waits across streams, for the previous step's (the warm start
// reads what it wrote, and consecutive back halves alternate their queue
// counters); that wait is for work submitted before, from this thread. The
// front half needs no order between steps: its stamps are numbered on the
// host, in submission order, and its scratch belongs to the buffer set's
// slot. A stage timed alone
// first waits for every other stream's work so far, and the next step waits
// for it.
static hipError_t submit_by_step(ov_pipe* p, long long t, int k, const double* poses, int64_t* count_out, int gen,
                                 bool reset, bool timed, bool alone) {
  hipStream_t s = p->st[k];
  hipError_t e = hipSuccess;
  p->ctx->hole_stamp = stamp_after(p->ctx->hole_stamp);
  const unsigned int stamp = p->ctx->hole_stamp;
  if (p->alone_pending) {
    e = hipStreamWaitEvent(s, p->alone_done, 0);
    p->alone_pending = false;
  }
  for (int stage = 0; stage < 3 && e == hipSuccess; ++stage) {
    if (stage == 2 && t >= 1) e = hipStreamWaitValue64(s, p->seq + 2, (uint64_t)t, hipStreamWaitValueGte, ~0ull);
    const bool ts = timed && stage == p->timed_stage;
    for (int g = 0; ts && alone && g < p->nsets && e == hipSuccess; ++g) {
      if (g == k) continue;
      e = hipEventRecord(p->join[g], p->st[g]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join[g], 0);
    }
    if (e == hipSuccess && ts) e = hipEventRecord(p->tb[p->ntimed], s);
    if (e == hipSuccess)
      e = stage_launch(p, k, stage, poses, s, stage == 2 ? (long long*)count_out : nullptr, gen, reset, stamp);
    if (e == hipSuccess && ts) e = hipEventRecord(p->te[p->ntimed], s);
    if (e == hipSuccess && ts && alone) {
      e = hipEventRecord(p->alone_done, s);
      p->alone_pending = e == hipSuccess;
    }
    if (e == hipSuccess && stage == 2) e = hipStreamWriteValue64(s, p->seq + 2, (uint64_t)(t + 1), 0);
  }
  return e;
}

int ov_pipe_submit(ov_pipe* p, const double* poses, int64_t* count_out) {
  if (!p || !poses) return pipe_fail(p, OV_EINVAL, "ov_pipe_submit: null argument");
  ov_ctx* ctx = p->ctx;
  const long long t = p->t;
  const int n = p->nsets;
  const int k = (int)(t % n);
  const ov_step_buffers& b = p->sets[k];
  hipError_t e = hipSuccess;
  const double* ps = poses;
  const bool timed = p->timing > 0 && (t - p->timing_t0) % p->timing == 0 && p->ntimed < (int)p->tb.size();
  const bool alone = timed && p->timed_alone;
  // alternate the slot's two near lists; from the set's second step on,
  // reset only the previous step's tiles (not under graphs, whose captured
  // launches cannot alternate)
  const long long use = p->uses[k]++;
  const int gen = p->graphs ? 0 : (int)(use & 1);
  const bool reset = !p->graphs && use > 0;
  p->gen[k] = gen;
  if (p->by_step) {
    e = submit_by_step(p, t, k, poses, count_out, gen, reset, timed, alone);
    if (e != hipSuccess) return hip_fail(ctx, e, "ov_pipe_submit");
    if (timed) ++p->ntimed;
    ++p->t;
    return OV_OK;
  }
  for (int g = 0; g < n && e == hipSuccess; ++g) {
    hipStream_t s = p->st[g];
    // after the previous group of this step, or (first group) after the
    // last group of the step that used this buffer set before
    const bool tg = timed && p->timed_stage >= first_stage(p, g) && p->timed_stage < first_stage(p, g + 1);
    const bool tg_alone = tg && alone;
    if (n > 1) {
      if (g > 0)
        e = hipStreamWaitValue64(s, p->seq + g - 1, (uint64_t)(t + 1), hipStreamWaitValueGte, ~0ull);
      else if (t >= n)
        e = hipStreamWaitValue64(s, p->seq + n - 1, (uint64_t)(t + 1 - n), hipStreamWaitValueGte, ~0ull);
      if (g == 0 && p->after_group >= 0 && e == hipSuccess) {
        e = hipStreamWaitValue64(s, p->seq + p->after_group, (uint64_t)p->after_value, hipStreamWaitValueGte, ~0ull);
        p->after_group = -1;
      }
      // a timed group also waits for the previous step's later groups, so
      // that its events time it alone
      for (int g2 = g + 1; tg_alone && g2 < n && t >= 1 && e == hipSuccess; ++g2)
        e = hipStreamWaitValue64(s, p->seq + g2, (uint64_t)t, hipStreamWaitValueGte, ~0ull);
      if (tg_alone) {
        p->after_group = g;
        p->after_value = t + 1;
      }
    }
    if (e == hipSuccess && g == 0 && p->graphs) {
      double* slot = p->poses_slot + 12 * ctx->grids.size() * k;
      e = hipMemcpyAsync(slot, poses, sizeof(double) * 12 * ctx->grids.size(), hipMemcpyDeviceToDevice, s);
      ps = slot;
    }
    if (p->graphs) {
      // (timing covers the whole graph of the timed stage's stream)
      if (e == hipSuccess && tg) e = hipEventRecord(p->tb[p->ntimed], s);
      if (e == hipSuccess) e = hipGraphLaunch(p->gx[k][g], s);
      if (e == hipSuccess && tg) e = hipEventRecord(p->te[p->ntimed], s);
      if (e == hipSuccess && g == n - 1 && count_out) e = launch_copy_count((long long*)count_out, b.d_count, s);
    } else {
      for (int stage = first_stage(p, g); stage < first_stage(p, g + 1) && e == hipSuccess; ++stage) {
        const bool ts = timed && stage == p->timed_stage;
        if (ts) e = hipEventRecord(p->tb[p->ntimed], s);
        if (e == hipSuccess)
          e = stage_launch(p, k, stage, ps, s, stage == 2 ? (long long*)count_out : nullptr, gen, reset);
        if (e == hipSuccess && ts) e = hipEventRecord(p->te[p->ntimed], s);
      }
    }
    if (e == hipSuccess && n > 1) e = hipStreamWriteValue64(s, p->seq + g, (uint64_t)(t + 1), 0);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "ov_pipe_submit");
  if (timed) ++p->ntimed;
  ++p->t;
  return OV_OK;
}

// submit_many with one host thread per stream: every step's bookkeeping
// (buffer set, near list, start kind, timing slot) is fixed first, in
// submission order; then thread g issues group g's waits, launches and
// counter writes for all the steps. The order between the groups is the
// device-side one of the counters; on the host a thread issues a wait only
// after the thread that writes the awaited counter has issued that write, so
// that, as with one thread, every wait is for work submitted before it (two
// streams that share a hardware queue could otherwise wait on each other).
// Each stream still receives its work in step order.
static int submit_threaded(ov_pipe* p, const double* poses, int64_t pose_stride, int64_t n, int64_t* counts_out) {
  struct Plan {
    long long t;
    int k, gen, tidx;
    bool reset;
    const double* poses;
    long long* count_out;
  };
  ov_ctx* ctx = p->ctx;
  const int ns = p->nsets;
  std::vector<Plan> plan((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    Plan& pl = plan[(size_t)i];
    pl.t = p->t + i;
    pl.k = (int)(pl.t % ns);
    const long long use = p->uses[pl.k]++;
    pl.gen = (int)(use & 1);
    pl.reset = use > 0;
    p->gen[pl.k] = pl.gen;
    const bool timed = p->timing > 0 && (pl.t - p->timing_t0) % p->timing == 0 && p->ntimed < (int)p->tb.size();
    pl.tidx = timed ? p->ntimed++ : -1;
    pl.poses = poses + pose_stride * i;
    pl.count_out = counts_out ? (long long*)(counts_out + i) : nullptr;
  }
  const int after_group = p->after_group;
  const long long after_value = p->after_value;
  p->after_group = -1;
  // issued[g]: the steps of this call whose group-g counter write is issued
  std::atomic<long long> issued[3];
  for (auto& v : issued) v.store(0);
  std::atomic<bool> failed{false};
  auto issued_at_least = [&](int g, long long steps) {
    while (issued[g].load(std::memory_order_acquire) < steps && !failed.load(std::memory_order_acquire))
      std::this_thread::yield();
    return !failed.load(std::memory_order_acquire);
  };
  auto run_group = [&](int g) -> hipError_t {
    hipError_t e = hipSetDevice(ctx->device);
    hipStream_t s = p->st[g];
    for (size_t i = 0; i < plan.size() && e == hipSuccess; ++i) {
      const Plan& pl = plan[i];
      if (g > 0) {
        if (!issued_at_least(g - 1, (long long)i + 1)) break;
        e = hipStreamWaitValue64(s, p->seq + g - 1, (uint64_t)(pl.t + 1), hipStreamWaitValueGte, ~0ull);
      } else if (pl.t >= ns) {
        // (a step of an earlier call was issued before this call began)
        if ((long long)i >= ns && !issued_at_least(ns - 1, (long long)i - ns + 1)) break;
        e = hipStreamWaitValue64(s, p->seq + ns - 1, (uint64_t)(pl.t + 1 - ns), hipStreamWaitValueGte, ~0ull);
      }
      if (g == 0 && i == 0 && after_group >= 0 && e == hipSuccess)
        e = hipStreamWaitValue64(s, p->seq + after_group, (uint64_t)after_value, hipStreamWaitValueGte, ~0ull);
      for (int stage = first_stage(p, g); stage < first_stage(p, g + 1) && e == hipSuccess; ++stage) {
        const bool ts = pl.tidx >= 0 && stage == p->timed_stage;
        if (ts) e = hipEventRecord(p->tb[pl.tidx], s);
        if (e == hipSuccess)
          e = stage_launch(p, pl.k, stage, pl.poses, s, stage == 2 ? pl.count_out : nullptr, pl.gen, pl.reset);
        if (e == hipSuccess && ts) e = hipEventRecord(p->te[pl.tidx], s);
      }
      if (e == hipSuccess) e = hipStreamWriteValue64(s, p->seq + g, (uint64_t)(pl.t + 1), 0);
      if (e == hipSuccess) issued[g].store((long long)i + 1, std::memory_order_release);
    }
    if (e != hipSuccess) failed.store(true, std::memory_order_release);
    return e;
  };
  std::vector<hipError_t> err((size_t)ns, hipSuccess);
  std::vector<std::thread> workers;
  for (int g = 1; g < ns; ++g) workers.emplace_back([&, g] { err[(size_t)g] = run_group(g); });
  err[0] = run_group(0);
  for (auto& w : workers) w.join();
  p->t += n;
  for (hipError_t e : err)
    if (e != hipSuccess) return hip_fail(ctx, e, "ov_pipe_submit_many");
  if (failed.load()) return pipe_fail(p, OV_EHIP, "ov_pipe_submit_many: a stream's thread stopped");
  return OV_OK;
}

int ov_pipe_set_by_step(ov_pipe* p, int32_t on) {
  if (!p || on < 0 || on > 1) return pipe_fail(p, OV_EINVAL, "ov_pipe_set_by_step: bad argument");
  if (p->t != 0) return pipe_fail(p, OV_ESTATE, "ov_pipe_set_by_step after the first submit");
  if (on && p->graphs) return pipe_fail(p, OV_ESTATE, "ov_pipe_set_by_step: not with graphs");
  if (on && p->nsets < 2) return pipe_fail(p, OV_EINVAL, "ov_pipe_set_by_step: needs two or three streams");
  if (on) {
    // the host numbers this pipe's stamps on from the device's step counter
    // (the context's earlier steps, whatever issued them, are done first)
    hipError_t e = hipDeviceSynchronize();
    unsigned int v = 0;
    if (e == hipSuccess) e = hipMemcpy(&v, p->ctx->d_stamp, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "ov_pipe_set_by_step");
    p->ctx->hole_stamp = v;
  }
  p->by_step = on != 0;
  return OV_OK;
}

int ov_pipe_set_threads(ov_pipe* p, int32_t on) {
  if (!p || on < 0 || on > 1) return pipe_fail(p, OV_EINVAL, "ov_pipe_set_threads: bad argument");
  p->threads = on != 0;
  return OV_OK;
}

int ov_pipe_submit_many(ov_pipe* p, const double* poses, int64_t pose_stride, int64_t n, int64_t* counts_out) {
  if (!p || !poses || n < 0 || pose_stride < 12 * (int64_t)p->ctx->grids.size())
    return pipe_fail(p, OV_EINVAL, "ov_pipe_submit_many: bad argument");
  if (p->threads && !p->by_step && p->nsets > 1 && !p->graphs && !(p->timing > 0 && p->timed_alone) && n > 1)
    return submit_threaded(p, poses, pose_stride, n, counts_out);
  for (int64_t i = 0; i < n; ++i) {
    int rc = ov_pipe_submit(p, poses + pose_stride * i, counts_out ? counts_out + i : nullptr);
    if (rc != OV_OK) return rc;
  }
  return OV_OK;
}

int ov_pipe_join(ov_pipe* p, void* stream) {
  if (!p) return OV_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (int g = 0; g < p->nsets && e == hipSuccess; ++g) {
    e = hipEventRecord(p->join[g], p->st[g]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join[g], 0);
  }
  return e == hipSuccess ? OV_OK : hip_fail(p->ctx, e, "ov_pipe_join");
}

int ov_pipe_stage_times(ov_pipe* p, float* ms_out, int32_t max, int32_t* n_out) {
  if (!p || !n_out || (max > 0 && !ms_out)) return OV_EINVAL;
  int n = p->ntimed < max ? p->ntimed : max;
  for (int i = 0; i < n; ++i) {
    hipError_t e = hipEventSynchronize(p->te[i]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_out[i], p->tb[i], p->te[i]);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "ov_pipe_stage_times");
  }
  *n_out = n;
  p->ntimed = 0;
  return OV_OK;
}

int ov_pipe_destroy(ov_pipe* p) {
  if (!p) return OV_EINVAL;
  for (int g = 0; g < p->nsets; ++g)
    if (p->st[g]) (void)hipStreamSynchronize(p->st[g]);
  destroy_graphs(p);
  for (int g = 0; g < 3; ++g)
    if (p->join[g]) (void)hipEventDestroy(p->join[g]);
  if (p->alone_done) (void)hipEventDestroy(p->alone_done);
  if (p->seq) (void)hipFree(p->seq);
  if (p->defer_items) (void)hipFree(p->defer_items);
  if (p->defer_count) (void)hipFree(p->defer_count);
  for (auto ev : p->tb)
    if (ev) (void)hipEventDestroy(ev);
  for (auto ev : p->te)
    if (ev) (void)hipEventDestroy(ev);
  delete p;
  return OV_OK;
}

}  // extern "C"
