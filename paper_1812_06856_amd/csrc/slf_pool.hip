// Rig pool of libslf (slf_pool_* in include/slf.h): rigs attached to one
// HBM budget and one stream, driven in stages.  A stage runs, for every
// active request, its next operation (the sweep or one refinement
// iteration); requests of the same operation and image format share one
// persistent launch over a device work queue.  slf_pool_step launches one
// stage, so requests submitted between steps join at the next stage
// boundary (continuous batching); slf_pool_run runs every active request to
// its end, optionally as a replayed HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "slf.h"
#include "slf_ctx.h"
#include "slf_internal.h"

using namespace slf;

namespace {

struct Req {
  slf_ctx *rig = nullptr;
  bool sweep = false;  // the sweep is still to run
  int next_iter = 1, end_iter = 1;  // iterations [next_iter, end_iter) still to run
  uint64_t tag = 0;
  bool finished() const { return !sweep && next_iter >= end_iter; }
};

struct Done {
  uint64_t tag;
  hipEvent_t ev;
};

// A group: the requests of one stage that run the same op in the same format.
struct Group {
  int op, fmt;
  std::vector<Req *> reqs;
};

constexpr int kStepSlots = 6;     // (op, format) groups in one step
constexpr int kGraphSlots = 64;   // groups in one replayed graph
constexpr int kRegions = 3;       // eager halves 0 and 1, then the graph region
constexpr int kSlots = 2 * kStepSlots + kGraphSlots;

int region_base(int r) { return r < 2 ? r * kStepSlots : 2 * kStepSlots; }

}  // namespace

struct slf_pool {
  int device = 0;
  hipStream_t own = nullptr, stream = nullptr;
  uint64_t budget = 0, used = 0;
  int n_cu = 0;
  int occ[2][3][3] = {};  // resident workgroups per CU by [op][format][level chunk 4/8/16]
  std::vector<slf_ctx *> rigs;
  std::vector<Req> active;
  std::vector<Done> done;
  slf_pool_config cfg;
  PoolStage *d_stages = nullptr, *h_stages = nullptr;
  int *d_counters = nullptr;
  float4 *d_parts = nullptr;  // level-part records of split sweeps
  int64_t parts_cap = 0, parts_fill = 0;
  hipEvent_t uploaded[kRegions] = {};
  int half = 0;
  hipGraphExec_t gexec = nullptr;
  std::vector<int> gsig;
  std::map<std::string, slf_pool_config> tuned;
  std::string err;

  int fail(int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
};

int slf_pool::fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  err = buf;
  return code;
}

namespace {

void default_config(slf_pool_config *c) {
  std::memset(c, 0, sizeof *c);
  c->struct_size = sizeof(slf_pool_config);
  c->sweep_level_chunk = 8;
  c->sweep_tile = 1;
  c->refine_tile = 1;
  c->blocks_per_cu = 0;
  c->use_graph = 1;
  c->sweep_level_split = 1;
}

int config_check(slf_pool *P, const slf_pool_config *c) {
  if (!c) return P->fail(SLF_EINVAL, "config is NULL");
  if (c->struct_size != (int)sizeof(slf_pool_config))
    return P->fail(SLF_EINVAL, "config struct_size %d, expected %d", c->struct_size, (int)sizeof(slf_pool_config));
  if (c->sweep_level_chunk != 4 && c->sweep_level_chunk != 8 && c->sweep_level_chunk != 16)
    return P->fail(SLF_EINVAL, "sweep_level_chunk must be 4, 8 or 16");
  if (c->sweep_tile < 1 || c->sweep_tile > 64 || c->refine_tile < 1 || c->refine_tile > 64)
    return P->fail(SLF_EINVAL, "tiles must be in [1, 64]");
  if (c->blocks_per_cu < 0 || c->blocks_per_cu > 64) return P->fail(SLF_EINVAL, "blocks_per_cu must be in [0, 64]");
  if (c->sweep_level_split < 1 || c->sweep_level_split > 16)
    return P->fail(SLF_EINVAL, "sweep_level_split must be in [1, 16]");
  return SLF_OK;
}

int chunk_index(int kc) { return kc == 4 ? 0 : kc == 16 ? 2 : 1; }

int blocks_for(const slf_pool *P, int op, int fmt) {
  const int occ = std::max(1, P->occ[op][fmt][chunk_index(P->cfg.sweep_level_chunk)]);
  const int per_cu = P->cfg.blocks_per_cu > 0 ? std::min(P->cfg.blocks_per_cu, occ) : occ;
  return per_cu * P->n_cu;
}

// Groups of the next stage of every unfinished request, in a fixed order
// (sweeps first, then formats ascending; requests in submission order).
std::vector<Group> plan_stage(std::vector<Req *> &reqs) {
  std::vector<Group> groups;
  for (int op = SLF_OP_SWEEP; op <= SLF_OP_REFINE; ++op)
    for (int fmt = SLF_IMAGE_U8; fmt <= SLF_IMAGE_F32; ++fmt) {
      Group g{op, fmt, {}};
      for (Req *r : reqs) {
        if (r->finished()) continue;
        const int rop = r->sweep ? SLF_OP_SWEEP : SLF_OP_REFINE;
        if (rop == op && r->rig->p.image_precision == fmt) g.reqs.push_back(r);
      }
      if (!g.reqs.empty()) groups.push_back(std::move(g));
    }
  return groups;
}

// Writes the stage table of one group (at most kPoolMaxJobs requests) and
// advances its requests.  s_cap limits the superpixels of every job (the
// autotuner's trials); 0 = all.
void fill_stage(slf_pool *P, PoolStage &st, const Group &g, int s_cap, bool advance) {
  const int tile = g.op == SLF_OP_SWEEP ? P->cfg.sweep_tile : P->cfg.refine_tile;
  const int split = g.op == SLF_OP_SWEEP ? P->cfg.sweep_level_split : 1;
  st.njobs = (int)g.reqs.size();
  st.tile = tile;
  st.pad = 0;
  st.parts = P->d_parts;
  int items = 0, sp = 0;
  for (int j = 0; j < st.njobs; ++j) {
    Req *r = g.reqs[j];
    PoolJob &J = st.jobs[j];
    std::memset(&J, 0, sizeof J);
    J.item_begin = items;
    J.S = s_cap > 0 ? std::min(r->rig->S, s_cap) : r->rig->S;
    J.split = split;
    J.sp_begin = sp;
    if (split > 1) {
      J.part_base = P->parts_fill;
      P->parts_fill += (int64_t)J.S * split;
    }
    sp += J.S;
    items += (J.S + tile - 1) / tile * split;
    // A job cut to its first s_cap claims (the autotuner's timing stages)
    // takes superpixels 0..J.S-1 in index order: its split-sweep part
    // records are reserved for J.S superpixels and addressed by superpixel,
    // and the rig's strip order would reach superpixels past J.S.
    const bool capped = J.S < r->rig->S;
    if (g.op == SLF_OP_SWEEP) {
      sweep_args(r->rig, J.sweep);
      if (capped) J.sweep.order = nullptr;
      if (advance) {
        after_sweep(r->rig);
        r->sweep = false;
      }
    } else {
      refine_args(r->rig, r->next_iter, J.refine);
      if (capped) J.refine.order = nullptr;
      if (advance) {
        after_refine(r->rig);
        ++r->next_iter;
      }
    }
  }
  st.total_sp = sp;
  for (int q = 0; q < kPoolQueues; ++q) {
    st.qbegin[q] = (int)((int64_t)items * q / kPoolQueues);
    st.qend[q] = (int)((int64_t)items * (q + 1) / kPoolQueues);
  }
}

// Waits until the last upload into region r has been consumed, so the
// pinned staging of the region may be rewritten.
int wait_region(slf_pool *P, int r) {
  if (hipEventSynchronize(P->uploaded[r]) != hipSuccess) return P->fail(SLF_EDEVICE, "hipEventSynchronize failed");
  return SLF_OK;
}

int upload(slf_pool *P, int r, int n) {
  const int base = region_base(r);
  if (hipMemcpyAsync(P->d_stages + base, P->h_stages + base, sizeof(PoolStage) * n, hipMemcpyHostToDevice,
                     P->stream) != hipSuccess ||
      hipEventRecord(P->uploaded[r], P->stream) != hipSuccess)
    return P->fail(SLF_EDEVICE, "stage table upload failed");
  return SLF_OK;
}

// Part records the sweep groups of `groups` need (split sweeps), grown
// before any stage table points at the buffer; in-flight work that may use
// the old buffer is waited for first.
int reserve_parts(slf_pool *P, const std::vector<Group> &groups, int s_cap) {
  P->parts_fill = 0;
  if (P->cfg.sweep_level_split <= 1) return SLF_OK;
  int64_t need = 0;
  for (const Group &g : groups)
    if (g.op == SLF_OP_SWEEP)
      for (const Req *r : g.reqs) need += (int64_t)(s_cap > 0 ? std::min(r->rig->S, s_cap) : r->rig->S);
  need *= P->cfg.sweep_level_split;
  if (need <= P->parts_cap) return SLF_OK;
  if (hipStreamSynchronize(P->stream) != hipSuccess) return P->fail(SLF_EDEVICE, "hipStreamSynchronize failed");
  if (P->d_parts) (void)hipFree(P->d_parts);
  P->d_parts = nullptr;
  P->parts_cap = 0;
  if (hipMalloc((void **)&P->d_parts, sizeof(float4) * need) != hipSuccess)
    return P->fail(SLF_ENOMEM, "pool part records: %lld bytes", (long long)(sizeof(float4) * need));
  P->parts_cap = need;
  return SLF_OK;
}

int launch_group(slf_pool *P, const Group &g, int slot) {
  const bool merge = g.op == SLF_OP_SWEEP && P->cfg.sweep_level_split > 1;
  const hipError_t e = launch_pool(g.op, g.fmt, P->cfg.sweep_level_chunk, merge, P->d_stages + slot,
                                   P->d_counters + slot * kPoolQueues * kPoolCounterStride,
                                   blocks_for(P, g.op, g.fmt), P->stream);
  if (e != hipSuccess) return P->fail(SLF_EDEVICE, "pooled launch: %s", hipGetErrorString(e));
  return SLF_OK;
}

// Completion of finished requests: an event on the pool stream that the
// rig's own stream waits for; poll reports the tag once it has fired.
int retire(slf_pool *P) {
  for (size_t i = 0; i < P->active.size();) {
    Req &r = P->active[i];
    if (!r.finished()) {
      ++i;
      continue;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, P->stream) != hipSuccess ||
        (r.rig->stream != P->stream && hipStreamWaitEvent(r.rig->stream, ev, 0) != hipSuccess))
      return P->fail(SLF_EDEVICE, "completion event failed");
    P->done.push_back({r.tag, ev});
    r.rig->in_flight = false;
    P->active.erase(P->active.begin() + i);
  }
  return SLF_OK;
}

int one_step(slf_pool *P) {
  std::vector<Req *> reqs;
  for (auto &r : P->active) reqs.push_back(&r);
  std::vector<Group> groups = plan_stage(reqs);
  if (groups.empty()) return retire(P);
  const int r = P->half;
  int rc;
  if ((rc = wait_region(P, r))) return rc;
  if ((rc = reserve_parts(P, groups, 0))) return rc;
  const int base = region_base(r);
  for (size_t i = 0; i < groups.size(); ++i) fill_stage(P, P->h_stages[base + i], groups[i], 0, true);
  if ((rc = upload(P, r, (int)groups.size()))) return rc;
  for (size_t i = 0; i < groups.size(); ++i)
    if ((rc = launch_group(P, groups[i], base + (int)i))) return rc;
  P->half ^= 1;
  return retire(P);
}

// Runs every active request to its end as one replayed HIP graph.  The graph
// holds, per group, the counter-reset kernel and the persistent kernel; the
// stage tables it reads live at fixed device addresses and are uploaded
// before each replay, so a graph serves any batch with the same stage shape.
int run_graph(slf_pool *P) {
  std::vector<Req *> reqs;
  for (auto &r : P->active) reqs.push_back(&r);
  // the whole schedule, stage by stage
  std::vector<Group> all;
  std::vector<int> sig;
  // a shadow run over the request fields only (rig state is untouched)
  const std::vector<Req> saved(P->active.begin(), P->active.end());
  for (;;) {
    std::vector<Group> groups = plan_stage(reqs);
    if (groups.empty()) break;
    for (auto &g : groups) {
      if (all.size() >= (size_t)kGraphSlots) {
        // too long for one graph: rewind and let the caller step eagerly
        for (size_t i = 0; i < reqs.size(); ++i) *reqs[i] = saved[i];
        return SLF_EUNSUPPORTED;
      }
      for (Req *r : g.reqs) {
        if (g.op == SLF_OP_SWEEP) r->sweep = false;
        else ++r->next_iter;
      }
      sig.push_back(g.op * 16 + g.fmt);
      all.push_back(g);
    }
    sig.push_back(-1);  // stage boundary
  }
  for (size_t i = 0; i < reqs.size(); ++i) *reqs[i] = saved[i];  // rewind the shadow run
  sig.push_back(P->cfg.sweep_level_chunk);
  sig.push_back(P->cfg.blocks_per_cu);
  sig.push_back(P->cfg.sweep_level_split);
  int rc;
  if ((rc = wait_region(P, 2))) return rc;
  if ((rc = reserve_parts(P, all, 0))) return rc;
  const int base = region_base(2);
  for (size_t i = 0; i < all.size(); ++i) fill_stage(P, P->h_stages[base + i], all[i], 0, true);
  if ((rc = upload(P, 2, (int)all.size()))) return rc;
  if (!P->gexec || P->gsig != sig) {
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    P->gexec = nullptr;
    P->gsig.clear();
    if (hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return P->fail(SLF_EDEVICE, "hipStreamBeginCapture failed");
    int lrc = SLF_OK;
    for (size_t i = 0; i < all.size() && !lrc; ++i) lrc = launch_group(P, all[i], base + (int)i);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(P->stream, &graph);
    if (lrc) {
      if (graph) (void)hipGraphDestroy(graph);
      return lrc;
    }
    if (ec != hipSuccess) return P->fail(SLF_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&P->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      P->gexec = nullptr;
      return P->fail(SLF_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    }
    P->gsig = sig;
  }
  if (hipGraphLaunch(P->gexec, P->stream) != hipSuccess) return P->fail(SLF_EDEVICE, "hipGraphLaunch failed");
  return retire(P);
}

std::string tune_key(const slf_pool *P) {
  std::vector<std::string> parts;
  for (const slf_ctx *c : P->rigs) {
    char b[96];
    snprintf(b, sizeof b, "%dx%d:%d:%d:%d:%d", c->vh[0].W, c->vh[0].H, (int)c->vh[0].nbrs.size(), c->p.levels,
             c->p.image_precision, c->V);
    parts.push_back(b);
  }
  std::sort(parts.begin(), parts.end());
  std::string k;
  for (auto &p : parts) k += p + ";";
  return k;
}

// Time of one stage over every attached rig (min of `reps`), capped at
// s_cap superpixels per rig; rig state is not advanced.
int time_stage(slf_pool *P, int op, int s_cap, int reps, float *ms) {
  std::vector<Req> tmp(P->rigs.size());
  std::vector<Req *> reqs;
  for (size_t i = 0; i < P->rigs.size(); ++i) {
    tmp[i].rig = P->rigs[i];
    tmp[i].sweep = op == SLF_OP_SWEEP;
    tmp[i].next_iter = 1;
    tmp[i].end_iter = op == SLF_OP_SWEEP ? 1 : 2;
    reqs.push_back(&tmp[i]);
  }
  std::vector<Group> groups = plan_stage(reqs);
  int rc;
  hipEvent_t t0, t1;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
    return P->fail(SLF_EDEVICE, "hipEventCreate failed");
  float best = 1e30f;
  for (int rep = 0; rep < reps; ++rep) {
    const int r = P->half;
    if ((rc = wait_region(P, r))) return rc;
    if ((rc = reserve_parts(P, groups, s_cap))) return rc;
    const int base = region_base(r);
    for (size_t i = 0; i < groups.size(); ++i) fill_stage(P, P->h_stages[base + i], groups[i], s_cap, false);
    if ((rc = upload(P, r, (int)groups.size()))) return rc;
    (void)hipEventRecord(t0, P->stream);
    for (size_t i = 0; i < groups.size(); ++i)
      if ((rc = launch_group(P, groups[i], base + (int)i))) return rc;
    (void)hipEventRecord(t1, P->stream);
    P->half ^= 1;
    if (hipEventSynchronize(t1) != hipSuccess) return P->fail(SLF_EDEVICE, "stage timing failed");
    float t = 0.f;
    (void)hipEventElapsedTime(&t, t0, t1);
    best = std::min(best, t);
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  *ms = best;
  return SLF_OK;
}

bool attached(const slf_pool *P, const slf_ctx *c) {
  return std::find(P->rigs.begin(), P->rigs.end(), c) != P->rigs.end();
}

}  // namespace

extern "C" {

void slf_pool_default_config(slf_pool_config *c) {
  if (c) default_config(c);
}

const char *slf_pool_last_error(const slf_pool *P) { return P ? P->err.c_str() : "pool is NULL"; }

int slf_pool_create(int device_ordinal, uint64_t hbm_budget_bytes, slf_pool **out) {
  if (!out) return SLF_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return SLF_EDEVICE;
  if (device_ordinal < 0 || device_ordinal >= n) return SLF_EINVAL;
  if (hipSetDevice(device_ordinal) != hipSuccess) return SLF_EDEVICE;
  slf_pool *P = new (std::nothrow) slf_pool();
  if (!P) return SLF_ENOMEM;
  P->device = device_ordinal;
  default_config(&P->cfg);
  size_t free_b = 0, total_b = 0;
  bool ok = hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
            hipDeviceGetAttribute(&P->n_cu, hipDeviceAttributeMultiprocessorCount, device_ordinal) == hipSuccess &&
            hipStreamCreateWithFlags(&P->own, hipStreamNonBlocking) == hipSuccess;
  P->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)total_b;
  for (int op = 0; op < 2; ++op)
    for (int fmt = 0; fmt < 3; ++fmt)
      for (int k = 0; k < 3; ++k) P->occ[op][fmt][k] = pool_occupancy(op, fmt, 4 << k);
  P->stream = P->own;
  ok = ok && hipMalloc((void **)&P->d_stages, sizeof(PoolStage) * kSlots) == hipSuccess &&
       hipHostMalloc((void **)&P->h_stages, sizeof(PoolStage) * kSlots, hipHostMallocDefault) == hipSuccess &&
       hipMalloc((void **)&P->d_counters, sizeof(int) * kSlots * kPoolQueues * kPoolCounterStride) == hipSuccess;
  for (int r = 0; r < kRegions && ok; ++r) {
    ok = hipEventCreateWithFlags(&P->uploaded[r], hipEventDisableTiming) == hipSuccess &&
         hipEventRecord(P->uploaded[r], P->stream) == hipSuccess;
  }
  if (!ok) {
    slf_pool_destroy(P);
    return SLF_ENOMEM;
  }
  std::memset(P->h_stages, 0, sizeof(PoolStage) * kSlots);
  *out = P;
  return SLF_OK;
}

int slf_pool_destroy(slf_pool *P) {
  if (!P) return SLF_EINVAL;
  (void)hipSetDevice(P->device);
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  for (auto &d : P->done) (void)hipEventDestroy(d.ev);
  for (slf_ctx *c : P->rigs) {
    c->pool = nullptr;
    c->pool_bytes = 0;
    c->in_flight = false;
  }
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  for (auto &e : P->uploaded)
    if (e) (void)hipEventDestroy(e);
  if (P->d_stages) (void)hipFree(P->d_stages);
  if (P->d_counters) (void)hipFree(P->d_counters);
  if (P->d_parts) (void)hipFree(P->d_parts);
  if (P->h_stages) (void)hipHostFree(P->h_stages);
  if (P->own) (void)hipStreamDestroy(P->own);
  delete P;
  return SLF_OK;
}

int slf_pool_set_stream(slf_pool *P, void *stream) {
  if (!P) return SLF_EINVAL;
  if (!P->active.empty()) return P->fail(SLF_ESTATE, "requests are active");
  (void)hipSetDevice(P->device);
  if (hipStreamSynchronize(P->stream) != hipSuccess) return P->fail(SLF_EDEVICE, "hipStreamSynchronize failed");
  P->stream = stream ? (hipStream_t)stream : P->own;
  for (auto &e : P->uploaded)
    if (hipEventRecord(e, P->stream) != hipSuccess) return P->fail(SLF_EDEVICE, "hipEventRecord failed");
  return SLF_OK;
}

int slf_pool_set_config(slf_pool *P, const slf_pool_config *cfg) {
  if (!P) return SLF_EINVAL;
  if (int rc = config_check(P, cfg)) return rc;
  if (!P->active.empty()) return P->fail(SLF_ESTATE, "requests are active");
  P->cfg = *cfg;
  return SLF_OK;
}

int slf_pool_get_config(slf_pool *P, slf_pool_config *cfg) {
  if (!P || !cfg) return SLF_EINVAL;
  *cfg = P->cfg;
  return SLF_OK;
}

int slf_pool_attach(slf_pool *P, slf_ctx *c) {
  if (!P || !c) return SLF_EINVAL;
  if (c->pool == P) return P->fail(SLF_ESTATE, "rig already attached");
  if (c->pool) return P->fail(SLF_ESTATE, "rig is attached to another pool");
  if (c->device != P->device) return P->fail(SLF_EINVAL, "rig is on device %d, pool on %d", c->device, P->device);
  if ((int)P->rigs.size() >= kPoolMaxJobs) return P->fail(SLF_EUNSUPPORTED, "at most %d rigs per pool", kPoolMaxJobs);
  uint64_t fp = 0;
  if (footprint(c, &fp)) return P->fail(SLF_ESTATE, "the rig's cameras and label grids must be set first");
  if (P->used + fp > P->budget)
    return P->fail(SLF_ENOMEM, "rig needs %llu bytes; %llu of %llu in use", (unsigned long long)fp,
                   (unsigned long long)P->used, (unsigned long long)P->budget);
  P->used += fp;
  c->pool = P;
  c->pool_bytes = fp;
  P->rigs.push_back(c);
  return SLF_OK;
}

int slf_pool_detach(slf_pool *P, slf_ctx *c) {
  if (!P || !c) return SLF_EINVAL;
  if (c->pool != P) return P->fail(SLF_EINVAL, "rig is not attached to this pool");
  if (c->in_flight) return P->fail(SLF_ESTATE, "rig has pool work not yet launched");
  P->used -= c->pool_bytes;
  c->pool = nullptr;
  c->pool_bytes = 0;
  P->rigs.erase(std::find(P->rigs.begin(), P->rigs.end(), c));
  return SLF_OK;
}

int slf_pool_usage(slf_pool *P, uint64_t *budget, uint64_t *used, int *n_rigs, int *n_active) {
  if (!P) return SLF_EINVAL;
  if (budget) *budget = P->budget;
  if (used) *used = P->used;
  if (n_rigs) *n_rigs = (int)P->rigs.size();
  if (n_active) *n_active = (int)P->active.size();
  return SLF_OK;
}

int slf_pool_submit(slf_pool *P, slf_ctx *c, int op, int first_iter, int n_iters, uint64_t tag) {
  if (!P || !c) return SLF_EINVAL;
  if (c->pool != P) return P->fail(SLF_EINVAL, "rig is not attached to this pool");
  if (c->in_flight) return P->fail(SLF_ESTATE, "rig already has a request in flight");
  if (op != SLF_POOL_SOLVE && op != SLF_POOL_PROPAGATE) return P->fail(SLF_EINVAL, "op must be SOLVE or PROPAGATE");
  if (first_iter < 1 || n_iters < 0) return P->fail(SLF_EINVAL, "need first_iter >= 1 and n_iters >= 0");
  if (hipSetDevice(P->device) != hipSuccess) return P->fail(SLF_EDEVICE, "hipSetDevice failed");
  uint64_t fp = 0;
  if (footprint(c, &fp)) return P->fail(SLF_ESTATE, "the rig's cameras and label grids must be set first");
  if (P->used - c->pool_bytes + fp > P->budget)
    return P->fail(SLF_ENOMEM, "rig grew to %llu bytes; over the pool budget", (unsigned long long)fp);
  if (int rc = ensure_setup(c)) return P->fail(rc, "rig setup: %s", c->err.c_str());
  P->used = P->used - c->pool_bytes + fp;
  c->pool_bytes = fp;
  if (op == SLF_POOL_PROPAGATE)
    for (const auto &v : c->vh)
      if (!v.has_planes) return P->fail(SLF_ESTATE, "every view of the rig needs planes before PROPAGATE");
  // the pool's stages start after everything already enqueued on the rig's stream
  if (c->stream != P->stream) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, c->stream) != hipSuccess ||
        hipStreamWaitEvent(P->stream, ev, 0) != hipSuccess)
      return P->fail(SLF_EDEVICE, "ordering against the rig's stream failed");
    (void)hipEventDestroy(ev);
  }
  Req r;
  r.rig = c;
  r.sweep = op == SLF_POOL_SOLVE;
  r.next_iter = first_iter;
  r.end_iter = first_iter + n_iters;
  r.tag = tag;
  c->in_flight = true;
  P->active.push_back(r);
  return SLF_OK;
}

int slf_pool_step(slf_pool *P, int *n_active) {
  if (!P) return SLF_EINVAL;
  if (hipSetDevice(P->device) != hipSuccess) return P->fail(SLF_EDEVICE, "hipSetDevice failed");
  int rc = one_step(P);
  if (n_active) *n_active = (int)P->active.size();
  return rc;
}

int slf_pool_run(slf_pool *P) {
  if (!P) return SLF_EINVAL;
  if (hipSetDevice(P->device) != hipSuccess) return P->fail(SLF_EDEVICE, "hipSetDevice failed");
  if (P->active.empty()) return SLF_OK;
  if (P->cfg.use_graph) {
    const int rc = run_graph(P);
    if (rc != SLF_EUNSUPPORTED) return rc;  // else: too many stages for one graph
  }
  while (!P->active.empty())
    if (int rc = one_step(P)) return rc;
  return SLF_OK;
}

int slf_pool_poll(slf_pool *P, uint64_t *tags, int max, int *n_done) {
  if (!P || !n_done || (max > 0 && !tags)) return SLF_EINVAL;
  *n_done = 0;
  for (size_t i = 0; i < P->done.size() && *n_done < max;) {
    const hipError_t e = hipEventQuery(P->done[i].ev);
    if (e == hipErrorNotReady) {
      ++i;
      continue;
    }
    if (e != hipSuccess) return P->fail(SLF_EDEVICE, "hipEventQuery: %s", hipGetErrorString(e));
    tags[(*n_done)++] = P->done[i].tag;
    (void)hipEventDestroy(P->done[i].ev);
    P->done.erase(P->done.begin() + i);
  }
  return SLF_OK;
}

int slf_pool_synchronize(slf_pool *P) {
  if (!P) return SLF_EINVAL;
  if (hipSetDevice(P->device) != hipSuccess || hipStreamSynchronize(P->stream) != hipSuccess)
    return P->fail(SLF_EDEVICE, "hipStreamSynchronize failed");
  return SLF_OK;
}

int slf_pool_autotune(slf_pool *P, int *from_cache) {
  if (!P) return SLF_EINVAL;
  if (from_cache) *from_cache = 0;
  if (!P->active.empty()) return P->fail(SLF_ESTATE, "requests are active");
  if (P->rigs.empty()) return P->fail(SLF_ESTATE, "no rigs attached");
  if (hipSetDevice(P->device) != hipSuccess) return P->fail(SLF_EDEVICE, "hipSetDevice failed");
  for (slf_ctx *c : P->rigs) {
    if (c->in_flight) return P->fail(SLF_ESTATE, "a rig has work in flight");
    if (int rc = ensure_setup(c)) return P->fail(rc, "rig setup: %s", c->err.c_str());
    if (c->stream != P->stream && hipStreamSynchronize(c->stream) != hipSuccess)
      return P->fail(SLF_EDEVICE, "hipStreamSynchronize failed");
  }
  const std::string key = tune_key(P);
  auto it = P->tuned.find(key);
  if (it != P->tuned.end()) {
    P->cfg = it->second;
    if (from_cache) *from_cache = 1;
    return SLF_OK;
  }
  // work counters and plane state are restored at the end
  std::vector<unsigned long long> work(kWorkCounters * P->rigs.size());
  std::vector<uint64_t> hwork(2 * P->rigs.size());
  for (size_t i = 0; i < P->rigs.size(); ++i) {
    slf_ctx *c = P->rigs[i];
    if (hipMemcpy(&work[kWorkCounters * i], c->d_work, kWorkCounters * sizeof(unsigned long long),
                  hipMemcpyDeviceToHost) != hipSuccess)
      return P->fail(SLF_EDEVICE, "work counter read failed");
    hwork[2 * i] = c->host_evals;
    hwork[2 * i + 1] = c->host_sweep_total;
  }
  const int s_cap = 2048;
  slf_pool_config best = P->cfg;
  float best_ms = 1e30f;
  int rc;
  for (int kc : {4, 8, 16})
    for (int tile : {1, 2})
      for (int split : {1, 2, 4}) {
        P->cfg.sweep_level_chunk = kc;
        P->cfg.sweep_tile = tile;
        P->cfg.sweep_level_split = split;
        float ms = 0.f;
        if ((rc = time_stage(P, SLF_OP_SWEEP, s_cap, 2, &ms))) return rc;
        if (ms < best_ms) {
          best_ms = ms;
          best.sweep_level_chunk = kc;
          best.sweep_tile = tile;
          best.sweep_level_split = split;
        }
      }
  P->cfg = best;
  // the refinement trials read a swept state
  {
    float ms = 0.f;
    if ((rc = time_stage(P, SLF_OP_SWEEP, 0, 1, &ms))) return rc;
  }
  best_ms = 1e30f;
  for (int tile : {1, 2, 4}) {
    P->cfg.refine_tile = tile;
    float ms = 0.f;
    if ((rc = time_stage(P, SLF_OP_REFINE, s_cap, 2, &ms))) return rc;
    if (ms < best_ms) {
      best_ms = ms;
      best.refine_tile = tile;
    }
  }
  P->cfg = best;
  // leave every rig as after a full sweep, with its counters as they were
  {
    float ms = 0.f;
    if ((rc = time_stage(P, SLF_OP_SWEEP, 0, 1, &ms))) return rc;
  }
  if (hipStreamSynchronize(P->stream) != hipSuccess) return P->fail(SLF_EDEVICE, "hipStreamSynchronize failed");
  for (size_t i = 0; i < P->rigs.size(); ++i) {
    slf_ctx *c = P->rigs[i];
    if (hipMemcpy(c->d_work, &work[kWorkCounters * i], kWorkCounters * sizeof(unsigned long long),
                  hipMemcpyHostToDevice) != hipSuccess)
      return P->fail(SLF_EDEVICE, "work counter restore failed");
    for (auto &v : c->vh) v.has_planes = true;
    c->host_evals = hwork[2 * i];
    c->host_sweep_total = hwork[2 * i + 1];
  }
  P->tuned[key] = best;
  return SLF_OK;
}

}  // extern "C"
