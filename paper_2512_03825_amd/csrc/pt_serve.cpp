// pt_serve.cpp -- served form of the parallel-tempering library: jobs arrive
// at any time, are admitted by device-memory budget, stay resident on the
// device, and advance together (continuous batching) until they finish.
#include "pt_arena.h"
#include "pt_host.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <thread>
#include <vector>

using namespace ptmi;

namespace {

constexpr uint32_t kMaxJobs = 65536;
constexpr uint32_t kMaxLanes = 8;
constexpr uint32_t kMaxDepth = 8;

struct Job {
  uint64_t id = 0;
  pt_config cfg{};
  std::vector<double> beta;
  uint64_t n_sweeps = 0;
  uint32_t every = 0, flags = 0;
  double arrival = 0, admitted = -1, finished = -1;
  size_t bytes = 0, off = 0;
  pt_ctx *ctx = nullptr;
  uint32_t lane = 0;
  uint32_t inst = ~0u;  // batched lane: instance slot
  uint64_t queued = 0;  // sweeps queued on the device so far
  bool done = false;
  // results, copied to the host when the job finishes
  std::vector<int32_t> E_slot, M_slot, Es, Ms;
  std::vector<uint32_t> wat, att, acc, bits;
  uint64_t sweeps_done = 0, exchanges_done = 0;
  uint32_t n_records = 0;

  ~Job() { pt_destroy(ctx); }
  uint64_t attempts() const { return (uint64_t)ctx_R() * ctx_N() * n_sweeps; }
  uint32_t ctx_R() const { return cfg.R; }
  uint64_t ctx_N() const {
    const uint64_t L = cfg.L;
    return cfg.model == PT_EA3D ? L * L * L : L * L;
  }
};

using Keep = std::vector<std::shared_ptr<std::vector<uint8_t>>>;

struct Step {
  hipEvent_t ev = nullptr;
  std::vector<uint64_t> finishing; // jobs whose last sweeps are in this step
  Keep keep;                       // host sources of uploads queued before it
};

struct Lane {
  hipStream_t s = nullptr;
  std::deque<Step> q;
  std::vector<uint64_t> jobs;  // tiled lanes: resident jobs in admission order
  Keep staged;                 // uploads queued since the last step
  uint64_t work = 0;           // tiled lanes: resident sites x replicas
};

struct Group {
  Geometry g;
  uint32_t W = 1, threads = 256, max_R = 0;
  uint32_t item_off = 0, n_items = 0;
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

template <class T>
std::shared_ptr<std::vector<uint8_t>> bytes_of(const T *p, size_t n) {
  auto v = std::make_shared<std::vector<uint8_t>>(n * sizeof(T));
  if (n) std::memcpy(v->data(), p, n * sizeof(T));
  return v;
}

struct Head {
  size_t insts, ctr, items, pairs, total;
};

Head head_layout(const pt_server_opts &o) {
  Head h;
  size_t off = 0;
  h.insts = off;
  off = align_up(off + (size_t)o.max_jobs * sizeof(BatchInst));
  h.ctr = off;
  off = align_up(off + (size_t)o.max_jobs * kCtrWords * 4);
  h.items = off;
  off = align_up(off + (size_t)std::max(o.max_walkers, 1u) * sizeof(BatchItem));
  h.pairs = off;
  off = align_up(off + (size_t)std::max(o.max_walkers, 1u) * sizeof(uint2));
  h.total = off;
  return h;
}

pt_status check_opts(const pt_server_opts *o) {
  if (!o) return fail(PT_EINVAL, "opts is NULL");
  if (o->max_jobs < 1 || o->max_jobs > kMaxJobs)
    return fail(PT_EINVAL, "max_jobs = %u: must be in [1, %u]", o->max_jobs, kMaxJobs);
  if (o->max_walkers < 1) return fail(PT_EINVAL, "max_walkers must be >= 1");
  if (o->tiled_lanes < 1 || o->tiled_lanes > kMaxLanes)
    return fail(PT_EINVAL, "tiled_lanes = %u: must be in [1, %u]", o->tiled_lanes, kMaxLanes);
  if (o->depth < 1 || o->depth > kMaxDepth)
    return fail(PT_EINVAL, "depth = %u: must be in [1, %u]", o->depth, kMaxDepth);
  if (o->cycle_sweeps < 1 || o->cycle_sweeps > 16)
    return fail(PT_EINVAL, "cycle_sweeps = %u: must be in [1, 16]", o->cycle_sweeps);
  if (o->tiled_sweeps < 1 || o->tiled_sweeps > 4096)
    return fail(PT_EINVAL, "tiled_sweeps = %u: must be in [1, 4096]", o->tiled_sweeps);
  return PT_OK;
}

}  // namespace

struct pt_server {
  pt_server_opts o{};
  uint8_t *base = nullptr;
  Head head{};
  BatchInst *d_insts = nullptr;
  uint32_t *d_ctr = nullptr;
  BatchItem *d_items = nullptr;
  uint2 *d_pairs = nullptr;
  uint8_t *arena_base = nullptr;
  Arena arena;
  std::vector<Lane> lanes; // [0] batched, [1 ..] tiled
  hipStream_t copy = nullptr;
  std::vector<hipEvent_t> event_pool;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> inst_job; // instance slot -> job id (0 = free)
  std::vector<uint32_t> free_inst;
  uint32_t inst_hi = 0;           // slots [0, inst_hi) have been used
  uint64_t walkers = 0;           // resident batched-lane replicas
  uint64_t resident = 0;
  bool members_dirty = true;
  std::vector<Group> groups;
  uint32_t n_pairs = 0;
  std::deque<pt_job_info> done_list;
  uint64_t next_id = 1, submitted = 0, finished = 0, attempts_finished = 0;
  uint64_t batched_cycles = 0, tiled_steps = 0;
  std::chrono::steady_clock::time_point t0;
  bool poisoned = false;
};

namespace {

pt_status sv_fail(pt_server *sv, hipError_t e, const char *what) {
  sv->poisoned = true;
  return fail(PT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

hipEvent_t take_event(pt_server *sv) {
  if (!sv->event_pool.empty()) {
    hipEvent_t e = sv->event_pool.back();
    sv->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Copy a finished job's observables to the host (copy stream, then wait).
hipError_t collect(pt_server *sv, Job &j) {
  pt_ctx *c = j.ctx;
  const size_t R = c->d.geo.R, N = c->d.geo.N;
  const DevState &st = c->st;
  hipError_t e = hipSuccess;
  auto D2H = [&](void *dst, const void *src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, sv->copy);
  };
  std::vector<int32_t> E(R), M(R);
  std::vector<uint32_t> flags(4), ctr(kCtrWords, 0u);
  j.wat.resize(R);
  j.att.resize(R);
  j.acc.resize(R);
  D2H(j.wat.data(), st.walker_at, R * 4);
  D2H(E.data(), st.E, R * 4);
  D2H(M.data(), st.M, R * 4);
  D2H(j.att.data(), st.att, R * 4);
  D2H(j.acc.data(), st.acc, R * 4);
  D2H(flags.data(), st.counter, 16);
  if (j.lane == 0) D2H(ctr.data(), sv->d_ctr + (size_t)j.inst * kCtrWords, kCtrWords * 4);
  j.n_records = records_between(c->cfg.record_every, 0, j.n_sweeps);
  j.Es.resize((size_t)j.n_records * R);
  j.Ms.resize((size_t)j.n_records * R);
  D2H(j.Es.data(), st.E_series, j.Es.size() * 4);
  D2H(j.Ms.data(), st.M_series, j.Ms.size() * 4);
  if (j.flags & PT_JOB_KEEP_SPINS) {
    j.bits.resize(R * N / 32);
    D2H(j.bits.data(), st.spins[c->cur], j.bits.size() * 4);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(sv->copy);
  if (e != hipSuccess) return e;
  j.sweeps_done = j.n_sweeps;
  j.exchanges_done = records_between(j.every, 0, j.n_sweeps);
  if (j.lane == 0 && (ctr[kCtrSweeps] != j.n_sweeps || ctr[kCtrExchanges] != j.exchanges_done ||
                      ctr[kCtrRecords] != j.n_records))
    return hipErrorUnknown;
  if (j.lane != 0 && (c->sweeps != j.n_sweeps || c->n_records != j.n_records)) return hipErrorUnknown;
  for (size_t k = 0; k < R; ++k)
    if (j.wat[k] >= R) return hipErrorUnknown;
  j.E_slot.resize(R);
  j.M_slot.resize(R);
  for (size_t k = 0; k < R; ++k) {
    j.E_slot[k] = E[j.wat[k]];
    j.M_slot[k] = M[j.wat[k]];
  }
  return hipSuccess;
}

pt_status retire(pt_server *sv, uint64_t id) {
  Job &j = *sv->jobs.at(id);
  if (collect(sv, j) != hipSuccess)
    return sv_fail(sv, hipErrorUnknown, "collecting a finished job's results");
  sv->arena.release(j.off, j.bytes);
  if (j.lane == 0) {
    sv->inst_job[j.inst] = 0;
    sv->free_inst.push_back(j.inst);
    sv->walkers -= j.cfg.R;
  } else {
    Lane &ln = sv->lanes[j.lane];
    ln.jobs.erase(std::find(ln.jobs.begin(), ln.jobs.end(), id));
    ln.work -= (uint64_t)j.cfg.R * j.ctx_N();
  }
  pt_destroy(j.ctx);
  j.ctx = nullptr;
  j.done = true;
  j.finished = now_s(sv->t0);
  --sv->resident;
  ++sv->finished;
  sv->attempts_finished += j.attempts();
  pt_job_info info{};
  info.job_id = id;
  info.arrival = j.arrival;
  info.admitted = j.admitted;
  info.finished = j.finished;
  info.attempts = j.attempts();
  info.lane = j.lane;
  sv->done_list.push_back(info);
  return PT_OK;
}

// Retire the jobs of every completed step at the head of each lane's queue.
pt_status drain_completed(pt_server *sv, uint32_t *n_ret) {
  for (Lane &ln : sv->lanes) {
    while (!ln.q.empty()) {
      const hipError_t q = hipEventQuery(ln.q.front().ev);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return sv_fail(sv, q, "step completion");
      Step st = std::move(ln.q.front());
      ln.q.pop_front();
      sv->event_pool.push_back(st.ev);
      for (uint64_t id : st.finishing) {
        pt_status s = retire(sv, id);
        if (s != PT_OK) return s;
        ++*n_ret;
      }
    }
  }
  return PT_OK;
}

// Admit queued jobs in arrival order while the head of the queue fits.
pt_status admit(pt_server *sv) {
  while (!sv->pending.empty()) {
    Job &j = *sv->jobs.at(sv->pending.front());
    const bool batched = j.lane == 0;
    if (sv->resident >= sv->o.max_jobs) break;
    if (batched && (sv->free_inst.empty() || sv->walkers + j.cfg.R > sv->o.max_walkers)) break;
    size_t off = 0;
    if (!sv->arena.alloc(j.bytes, &off)) break;
    sv->pending.pop_front();
    j.off = off;
    Lane *ln = &sv->lanes[0];
    if (!batched) {
      // the tiled lane with the least resident work
      uint32_t best = 1;
      for (uint32_t l = 2; l < sv->lanes.size(); ++l)
        if (sv->lanes[l].work < sv->lanes[best].work) best = l;
      j.lane = best;
      ln = &sv->lanes[best];
    }
    pt_status s = ctx_create(&j.cfg, ln->s, sv->arena_base + off, j.bytes, false, &j.ctx);
    if (s != PT_OK) {
      sv->poisoned = true;
      return s;
    }
    if (!batched && j.ctx->d.geo.dim == 2) {
      // Tiled lanes run several jobs at once, so a job's own grid need not
      // fill the chip: tall tiles (fewest recomputed halo rows) and 5 sweeps
      // per launch; the context's automatic plan stays if this one is invalid.
      pt_plan p{};
      p.mode = PT_PLAN_TILED;
      p.tile_planes = std::min<uint32_t>(j.ctx->d.geo.L, 256u);
      p.sweeps_per_launch = 5;
      p.block_threads = p.tile_planes >= 256u ? 1024u : 512u;
      (void)pt_set_plan(j.ctx, &p);
    }
    j.admitted = now_s(sv->t0);
    ++sv->resident;
    if (batched) {
      j.inst = sv->free_inst.back();
      sv->free_inst.pop_back();
      sv->inst_job[j.inst] = j.id;
      sv->inst_hi = std::max(sv->inst_hi, j.inst + 1u);
      sv->walkers += j.cfg.R;
      const BatchInst I = batch_inst(j.ctx, sv->d_ctr + (size_t)j.inst * kCtrWords);
      uint32_t ctr[kCtrWords] = {0u};
      ctr[kCtrTarget] = (uint32_t)j.n_sweeps;
      ctr[kCtrActive] = 1u;
      ctr[kCtrEvery] = j.every;
      auto hi = bytes_of(&I, 1), hc = bytes_of(ctr, kCtrWords);
      hipError_t e = hipMemcpyAsync(sv->d_insts + j.inst, hi->data(), hi->size(), hipMemcpyHostToDevice, ln->s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(sv->d_ctr + (size_t)j.inst * kCtrWords, hc->data(), hc->size(),
                           hipMemcpyHostToDevice, ln->s);
      if (e != hipSuccess) return sv_fail(sv, e, "job admission");
      ln->staged.push_back(hi);
      ln->staged.push_back(hc);
      sv->members_dirty = true;
    } else {
      ln->jobs.push_back(j.id);
      ln->work += (uint64_t)j.cfg.R * j.ctx_N();
    }
  }
  return PT_OK;
}

// Rebuild the batched lane's work lists from the resident, unfinished jobs.
pt_status rebuild_members(pt_server *sv) {
  Lane &ln = sv->lanes[0];
  std::map<std::pair<uint32_t, uint32_t>, std::vector<uint64_t>> by_geo;
  for (uint32_t i = 0; i < sv->inst_hi; ++i) {
    const uint64_t id = sv->inst_job[i];
    if (!id) continue;
    Job &j = *sv->jobs.at(id);
    if (j.queued >= j.n_sweeps) continue;
    by_geo[{j.ctx->d.geo.dim, j.ctx->d.geo.L}].push_back(id);
  }
  std::vector<BatchItem> items;
  std::vector<uint2> pairs;
  sv->groups.clear();
  for (auto &kv : by_geo) {
    Group G;
    G.g = sv->jobs.at(kv.second[0])->ctx->d.geo;
    for (uint64_t id : kv.second) G.max_R = std::max(G.max_R, sv->jobs.at(id)->cfg.R);
    const auto wt = batch_decomposition(G.g, G.max_R);
    G.W = wt.first;
    G.threads = wt.second;
    G.item_off = (uint32_t)items.size();
    for (uint64_t id : kv.second) {
      const Job &j = *sv->jobs.at(id);
      for (uint32_t w0 = 0; w0 < j.cfg.R; w0 += G.W) items.push_back({j.inst, w0});
      for (uint32_t k = 0; k + 1 < j.cfg.R; ++k) pairs.push_back(make_uint2(j.inst, k));
    }
    G.n_items = (uint32_t)items.size() - G.item_off;
    sv->groups.push_back(G);
  }
  // largest lattices first, so the longest workgroups start first
  std::sort(sv->groups.begin(), sv->groups.end(), [](const Group &x, const Group &y) {
    return x.g.N * (x.g.dim == 3 ? 4u : 1u) > y.g.N * (y.g.dim == 3 ? 4u : 1u);
  });
  sv->n_pairs = (uint32_t)pairs.size();
  hipError_t e = hipSuccess;
  if (!items.empty()) {
    auto hv = bytes_of(items.data(), items.size());
    e = hipMemcpyAsync(sv->d_items, hv->data(), hv->size(), hipMemcpyHostToDevice, ln.s);
    ln.staged.push_back(hv);
  }
  if (e == hipSuccess && !pairs.empty()) {
    auto hv = bytes_of(pairs.data(), pairs.size());
    e = hipMemcpyAsync(sv->d_pairs, hv->data(), hv->size(), hipMemcpyHostToDevice, ln.s);
    ln.staged.push_back(hv);
  }
  if (e != hipSuccess) return sv_fail(sv, e, "batched work lists");
  sv->members_dirty = false;
  return PT_OK;
}

// Queue one cycle of the batched lane; false if it has nothing to run.
pt_status batched_cycle(pt_server *sv, bool *queued) {
  *queued = false;
  if (sv->members_dirty) {
    pt_status s = rebuild_members(sv);
    if (s != PT_OK) return s;
  }
  if (sv->groups.empty()) return PT_OK;
  Lane &ln = sv->lanes[0];
  const uint32_t K = sv->o.cycle_sweeps;
  hipError_t e = hipSuccess;
  for (const Group &G : sv->groups)
    if (e == hipSuccess)
      e = launch_batch_sweep(sv->d_insts, sv->d_items + G.item_off, G.n_items, G.g, G.W, G.threads, K, ln.s);
  if (e == hipSuccess && sv->n_pairs) e = launch_batch_exchange(sv->d_insts, sv->d_pairs, sv->n_pairs, K, ln.s);
  if (e == hipSuccess) e = launch_batch_advance(sv->d_insts, sv->inst_hi, K, ln.s);
  if (e != hipSuccess) return sv_fail(sv, e, "batched cycle launch");
  Step st;
  // the device's schedule of this cycle, replayed on the host
  for (uint32_t i = 0; i < sv->inst_hi; ++i) {
    const uint64_t id = sv->inst_job[i];
    if (!id) continue;
    Job &j = *sv->jobs.at(id);
    if (j.queued >= j.n_sweeps) continue;
    uint64_t n = std::min<uint64_t>(K, j.n_sweeps - j.queued);
    if (j.every) n = std::min<uint64_t>(n, j.every - j.queued % j.every);
    j.queued += n;
    if (j.queued == j.n_sweeps) {
      st.finishing.push_back(id);
      sv->members_dirty = true;
    }
  }
  st.ev = take_event(sv);
  if (!st.ev) return sv_fail(sv, hipErrorOutOfMemory, "event creation");
  if ((e = hipEventRecord(st.ev, ln.s)) != hipSuccess) return sv_fail(sv, e, "step event");
  st.keep = std::move(ln.staged);
  ln.staged.clear();
  ln.q.push_back(std::move(st));
  ++sv->batched_cycles;
  *queued = true;
  return PT_OK;
}

// Queue one step of a tiled lane: every resident job there advances by up to
// tiled_sweeps sweeps.
pt_status tiled_step(pt_server *sv, uint32_t l, bool *queued) {
  *queued = false;
  Lane &ln = sv->lanes[l];
  Step st;
  bool any = false;
  for (uint64_t id : ln.jobs) {
    Job &j = *sv->jobs.at(id);
    if (j.queued >= j.n_sweeps) continue;
    const uint32_t n = (uint32_t)std::min<uint64_t>(sv->o.tiled_sweeps, j.n_sweeps - j.queued);
    pt_status s = ctx_advance(j.ctx, n, j.every);
    if (s != PT_OK) {
      sv->poisoned = true;
      return s;
    }
    j.queued += n;
    any = true;
    if (j.queued == j.n_sweeps) st.finishing.push_back(id);
  }
  if (!any) return PT_OK;
  st.ev = take_event(sv);
  if (!st.ev) return sv_fail(sv, hipErrorOutOfMemory, "event creation");
  hipError_t e = hipEventRecord(st.ev, ln.s);
  if (e != hipSuccess) return sv_fail(sv, e, "step event");
  st.keep = std::move(ln.staged);
  ln.staged.clear();
  ln.q.push_back(std::move(st));
  ++sv->tiled_steps;
  *queued = true;
  return PT_OK;
}

pt_status top_up(pt_server *sv, bool *queued_any) {
  *queued_any = false;
  for (uint32_t l = 0; l < sv->lanes.size(); ++l) {
    while (sv->lanes[l].q.size() < sv->o.depth) {
      bool q = false;
      pt_status s = l == 0 ? batched_cycle(sv, &q) : tiled_step(sv, l, &q);
      if (s != PT_OK) return s;
      if (!q) break;
      *queued_any = true;
    }
  }
  return PT_OK;
}

}  // namespace

extern "C" {

size_t pt_server_overhead_bytes(const pt_server_opts *opts) {
  if (check_opts(opts) != PT_OK) return 0;
  return head_layout(*opts).total;
}

pt_status pt_server_create(const pt_server_opts *opts, void *d_workspace, size_t ws_bytes,
                           pt_server **out) {
  if (!out) return fail(PT_EINVAL, "out is NULL");
  *out = nullptr;
  pt_status s = check_opts(opts);
  if (s != PT_OK) return s;
  if (!d_workspace || (uintptr_t)d_workspace % kAlign) return fail(PT_EINVAL, "workspace must be 256-byte aligned");
  const Head h = head_layout(*opts);
  if (ws_bytes <= h.total) return fail(PT_ENOMEM, "workspace of %zu bytes, the tables alone need %zu", ws_bytes, h.total);
  pt_server *sv = new (std::nothrow) pt_server();
  if (!sv) return fail(PT_ENOMEM, "host allocation failed");
  sv->o = *opts;
  sv->base = (uint8_t *)d_workspace;
  sv->head = h;
  sv->d_insts = (BatchInst *)(sv->base + h.insts);
  sv->d_ctr = (uint32_t *)(sv->base + h.ctr);
  sv->d_items = (BatchItem *)(sv->base + h.items);
  sv->d_pairs = (uint2 *)(sv->base + h.pairs);
  sv->arena_base = sv->base + h.total;
  sv->arena.reset(ws_bytes - h.total, kAlign);
  sv->inst_job.assign(opts->max_jobs, 0);
  for (uint32_t i = opts->max_jobs; i-- > 0;) sv->free_inst.push_back(i);
  sv->lanes.resize(1 + opts->tiled_lanes);
  hipError_t e = hipSuccess;
  for (Lane &ln : sv->lanes)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ln.s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->copy, hipStreamNonBlocking);
  // every instance slot starts idle, with a valid counter pointer
  std::vector<BatchInst> insts(opts->max_jobs);
  std::memset(insts.data(), 0, insts.size() * sizeof(BatchInst));
  for (uint32_t i = 0; i < opts->max_jobs; ++i) insts[i].ctr = sv->d_ctr + (size_t)i * kCtrWords;
  std::vector<uint32_t> zeros((size_t)opts->max_jobs * kCtrWords, 0u);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sv->d_insts, insts.data(), insts.size() * sizeof(BatchInst), hipMemcpyHostToDevice, sv->lanes[0].s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sv->d_ctr, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice, sv->lanes[0].s);
  if (e == hipSuccess) e = hipStreamSynchronize(sv->lanes[0].s);
  if (e != hipSuccess) {
    pt_server_destroy(sv);
    return fail(PT_EDEVICE, "server initialisation: %s", hipGetErrorString(e));
  }
  sv->t0 = std::chrono::steady_clock::now();
  *out = sv;
  return PT_OK;
}

pt_status pt_server_submit(pt_server *sv, const pt_config *cfg, uint64_t n_sweeps,
                           uint32_t exchange_every, uint32_t flags, double arrival,
                           uint64_t *job_id) {
  if (!sv) return fail(PT_EINVAL, "server is NULL");
  if (sv->poisoned) return fail(PT_ESTATE, "server is poisoned by an earlier device error");
  if (!cfg) return fail(PT_EINVAL, "config is NULL");
  if (cfg->init_spins || cfg->couplings)
    return fail(PT_EINVAL, "served jobs draw their spins and couplings from their seeds (no uploads)");
  if (n_sweeps < 1 || n_sweeps > 0xFFFFFFFFull)
    return fail(PT_EINVAL, "n_sweeps = %llu: must be in [1, 2^32 - 1]", (unsigned long long)n_sweeps);
  if (flags & ~PT_JOB_KEEP_SPINS) return fail(PT_EINVAL, "unknown flags 0x%x", flags);
  const size_t bytes = pt_workspace_bytes(cfg);
  if (!bytes) return PT_EINVAL; // message set by the configuration check
  if (cfg->record_every && records_between(cfg->record_every, 0, n_sweeps) > cfg->max_records)
    return fail(PT_EINVAL, "%u records would exceed max_records = %u",
                records_between(cfg->record_every, 0, n_sweeps), cfg->max_records);
  if (!sv->arena.could_fit(bytes))
    return fail(PT_ENOMEM, "job needs %zu bytes, the arena holds %zu", bytes, sv->arena.size());
  auto j = std::make_unique<Job>();
  j->id = sv->next_id++;
  j->cfg = *cfg;
  j->beta.assign(cfg->beta, cfg->beta + cfg->R);
  j->cfg.beta = j->beta.data();
  j->n_sweeps = n_sweeps;
  j->every = exchange_every;
  j->flags = flags;
  j->arrival = arrival < 0 ? now_s(sv->t0) : arrival;
  j->bytes = bytes;
  const uint32_t dim = cfg->model == PT_EA3D ? 3u : 2u;
  Geometry g{};
  g.dim = dim;
  g.L = cfg->L;
  g.R = cfg->R;
  g.N = cfg->L * cfg->L * (dim == 3 ? cfg->L : 1u);
  j->lane = batch_fits(g) ? 0u : 1u;
  if (j->lane == 0 && cfg->R > sv->o.max_walkers)
    return fail(PT_ENOMEM, "job has %u replicas, the batched lane holds %u", cfg->R, sv->o.max_walkers);
  if (job_id) *job_id = j->id;
  sv->pending.push_back(j->id);
  sv->jobs[j->id] = std::move(j);
  ++sv->submitted;
  return PT_OK;
}

pt_status pt_server_step(pt_server *sv, uint32_t wait_us, uint32_t *n_finished) {
  if (n_finished) *n_finished = 0;
  if (!sv) return fail(PT_EINVAL, "server is NULL");
  if (sv->poisoned) return fail(PT_ESTATE, "server is poisoned by an earlier device error");
  uint32_t n = 0;
  pt_status s = drain_completed(sv, &n);
  if (s == PT_OK) s = admit(sv);
  bool queued = false;
  if (s == PT_OK) s = top_up(sv, &queued);
  if (s != PT_OK) return s;
  if (n == 0 && wait_us) {
    bool inflight = false;
    for (const Lane &ln : sv->lanes) inflight |= !ln.q.empty();
    const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(wait_us);
    while (inflight && n == 0 && std::chrono::steady_clock::now() < until) {
      bool ready = false;
      for (const Lane &ln : sv->lanes)
        if (!ln.q.empty() && hipEventQuery(ln.q.front().ev) != hipErrorNotReady) ready = true;
      if (!ready) {
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        continue;
      }
      s = drain_completed(sv, &n);
      if (s == PT_OK) s = admit(sv);
      if (s == PT_OK) s = top_up(sv, &queued);
      if (s != PT_OK) return s;
      inflight = false;
      for (const Lane &ln : sv->lanes) inflight |= !ln.q.empty();
    }
  }
  if (n_finished) *n_finished = n;
  return PT_OK;
}

pt_status pt_server_done(pt_server *sv, pt_job_info *out, uint32_t cap, uint32_t *n) {
  if (!sv || !n || (cap && !out)) return fail(PT_EINVAL, "NULL argument");
  uint32_t k = 0;
  while (k < cap && !sv->done_list.empty()) {
    out[k++] = sv->done_list.front();
    sv->done_list.pop_front();
  }
  *n = k;
  return PT_OK;
}

pt_status pt_server_result(const pt_server *sv, uint64_t job_id, pt_obs *obs) {
  if (!sv || !obs) return fail(PT_EINVAL, "NULL argument");
  auto it = sv->jobs.find(job_id);
  if (it == sv->jobs.end()) return fail(PT_EINVAL, "no job %llu", (unsigned long long)job_id);
  const Job &j = *it->second;
  if (!j.done) return fail(PT_ESTATE, "job %llu has not finished", (unsigned long long)job_id);
  const size_t R = j.cfg.R, N = j.ctx_N();
  if (obs->spins && !(j.flags & PT_JOB_KEEP_SPINS))
    return fail(PT_EINVAL, "job %llu was submitted without PT_JOB_KEEP_SPINS", (unsigned long long)job_id);
  if (obs->spins && obs->spins_slot != PT_ALL_SLOTS && obs->spins_slot >= R)
    return fail(PT_EINVAL, "spins_slot = %u out of range", obs->spins_slot);
  if (obs->E_series) std::memcpy(obs->E_series, j.Es.data(), j.Es.size() * 4);
  if (obs->M_series) std::memcpy(obs->M_series, j.Ms.data(), j.Ms.size() * 4);
  if (obs->walker_at) std::memcpy(obs->walker_at, j.wat.data(), R * 4);
  if (obs->E_slot) std::memcpy(obs->E_slot, j.E_slot.data(), R * 4);
  if (obs->M_slot) std::memcpy(obs->M_slot, j.M_slot.data(), R * 4);
  if (obs->swap_att) std::memset(obs->swap_att, 0, R * R * 8);
  if (obs->swap_acc) std::memset(obs->swap_acc, 0, R * R * 8);
  for (size_t k = 0; k + 1 < R; ++k) {
    if (obs->swap_att) obs->swap_att[k * R + k + 1] = obs->swap_att[(k + 1) * R + k] = j.att[k];
    if (obs->swap_acc) obs->swap_acc[k * R + k + 1] = obs->swap_acc[(k + 1) * R + k] = j.acc[k];
  }
  if (obs->spins) {
    const size_t wpr = N / 32;
    auto unpack = [&](size_t w, int8_t *dst) {
      const uint32_t *src = j.bits.data() + w * wpr;
      for (size_t i = 0; i < N; ++i) dst[i] = ((src[i >> 5] >> (i & 31)) & 1u) ? -1 : 1;
    };
    if (obs->spins_slot == PT_ALL_SLOTS)
      for (size_t k = 0; k < R; ++k) unpack(j.wat[k], obs->spins + k * N);
    else
      unpack(j.wat[obs->spins_slot], obs->spins);
  }
  obs->sweeps_done = j.sweeps_done;
  obs->exchanges_done = j.exchanges_done;
  obs->n_records = j.n_records;
  return PT_OK;
}

pt_status pt_server_release(pt_server *sv, uint64_t job_id) {
  if (!sv) return fail(PT_EINVAL, "server is NULL");
  auto it = sv->jobs.find(job_id);
  if (it == sv->jobs.end()) return fail(PT_EINVAL, "no job %llu", (unsigned long long)job_id);
  if (!it->second->done) return fail(PT_ESTATE, "job %llu has not finished", (unsigned long long)job_id);
  sv->jobs.erase(it);
  return PT_OK;
}

pt_status pt_server_stats_get(const pt_server *sv, pt_server_stats *out) {
  if (!sv || !out) return fail(PT_EINVAL, "NULL argument");
  out->submitted = sv->submitted;
  out->pending = sv->pending.size();
  out->resident = sv->resident;
  out->finished = sv->finished;
  out->arena_bytes = sv->arena.size();
  out->arena_used = sv->arena.used();
  out->arena_peak = sv->arena.peak();
  out->walkers_resident = sv->walkers;
  out->batched_cycles = sv->batched_cycles;
  out->tiled_steps = sv->tiled_steps;
  out->attempts_finished = sv->attempts_finished;
  return PT_OK;
}

double pt_server_clock(const pt_server *sv) { return sv ? now_s(sv->t0) : 0.0; }

void pt_server_destroy(pt_server *sv) {
  if (!sv) return;
  for (Lane &ln : sv->lanes)
    if (ln.s) (void)hipStreamSynchronize(ln.s);
  if (sv->copy) (void)hipStreamSynchronize(sv->copy);
  for (Lane &ln : sv->lanes) {
    for (Step &st : ln.q)
      if (st.ev) (void)hipEventDestroy(st.ev);
    if (ln.s) (void)hipStreamDestroy(ln.s);
  }
  for (hipEvent_t e : sv->event_pool) (void)hipEventDestroy(e);
  if (sv->copy) (void)hipStreamDestroy(sv->copy);
  sv->jobs.clear();
  delete sv;
}

}  // extern "C"
