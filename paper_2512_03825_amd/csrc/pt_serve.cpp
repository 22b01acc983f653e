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
constexpr size_t kTiledLds = 144u * 1024u; // LDS budget of a tiled-lane workgroup

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
  uint32_t inst = ~0u;  // instance slot (device descriptor and counters)
  uint32_t tiles = 0;   // tiled lanes: tiles per walker (0: a batched-lane job)
  uint32_t cur = 0;     // tiled lanes: spin buffer holding the lattices (host replay)
  uint64_t queued = 0;  // sweeps queued on the device so far
  bool done = false;
  // results, copied to the host when the job finishes
  std::vector<int32_t> E_slot, M_slot, Es, Ms;
  std::vector<uint32_t> wat, att, acc, bits;
  uint64_t sweeps_done = 0, exchanges_done = 0;
  uint32_t n_records = 0;

  ~Job() { pt_destroy(ctx); }
  uint64_t attempts() const { return (uint64_t)cfg.R * sites() * n_sweeps; }
  uint64_t sites() const {
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

// A launch group of a lane: jobs of one lattice geometry.
struct Group {
  Geometry g;
  uint32_t W = 1, threads = 256, max_R = 0; // batched lane: walkers per workgroup
  uint32_t H = 0;                           // tiled lanes: rows per tile
  uint32_t item_off = 0, n_items = 0;
};

// A lane is a stream with its own resident jobs and device work lists: the
// batched lanes run whole-replica jobs through the batched kernels (lane 0 for
// lattices above every size class, then one lane per class after the tiled
// lanes), the tiled lanes (1 .. tiled_lanes) run larger lattices through the
// batched tiled kernel.
struct Lane {
  bool tiled = false;
  hipStream_t s = nullptr;
  std::deque<Step> q;
  std::vector<uint64_t> jobs;  // resident jobs in admission order
  Keep staged;                 // uploads queued since the last step
  bool dirty = true;           // membership changed since the lists were built
  uint64_t slots = 0;          // resident walkers (batched) or walker tiles (tiled lanes)
  uint64_t work = 0;           // resident sites x replicas
  uint32_t K = 1;              // sweeps per cycle
  std::vector<Group> groups;
  uint32_t n_pairs = 0, n_list = 0;
  // device work lists in the server's tables
  BatchItem *d_items = nullptr;      // batched lanes
  BatchTileItem *d_titems = nullptr; // tiled lanes
  uint2 *d_pairs = nullptr;          // batched lanes
  uint32_t *d_list = nullptr;        // instances the lane advances
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

// Server tables at the head of the workspace: instance descriptors and
// counters, then per lane its work lists (each sized by max_walkers entries
// and max_jobs instances).
struct Head {
  size_t insts, ctr, total;
  std::vector<size_t> items, pairs, list; // per lane
};

// Size classes of the batched lanes: the nonzero entries of class_sites.
uint32_t n_classes(const pt_server_opts &o) {
  uint32_t n = 0;
  while (n < PT_SERVER_CLASSES && o.class_sites[n]) ++n;
  return n;
}
uint32_t n_lanes(const pt_server_opts &o) { return 1u + o.tiled_lanes + n_classes(o); }
bool lane_tiled(const pt_server_opts &o, uint32_t l) { return l >= 1u && l <= o.tiled_lanes; }

Head head_layout(const pt_server_opts &o) {
  Head h;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t W = std::max(o.max_walkers, 1u);
  h.insts = take((size_t)o.max_jobs * sizeof(BatchInst));
  h.ctr = take((size_t)o.max_jobs * kCtrWords * 4);
  for (uint32_t l = 0; l < n_lanes(o); ++l) {
    const bool tiled = lane_tiled(o, l);
    h.items.push_back(take(W * (tiled ? sizeof(BatchTileItem) : sizeof(BatchItem))));
    h.pairs.push_back(tiled ? 0 : take(W * sizeof(uint2)));
    h.list.push_back(take((size_t)o.max_jobs * 4));
  }
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
  if (o->tiled_sweeps < 1 || o->tiled_sweeps > kMaxSweepsPerLaunch)
    return fail(PT_EINVAL, "tiled_sweeps = %u: must be in [1, %u]", o->tiled_sweeps,
                kMaxSweepsPerLaunch);
  const uint32_t nc = n_classes(*o);
  for (uint32_t k = 0; k < PT_SERVER_CLASSES; ++k) {
    if (k >= nc && o->class_sites[k])
      return fail(PT_EINVAL, "class_sites[%u] = %u after a zero entry", k, o->class_sites[k]);
    if (k > 0 && k < nc && o->class_sites[k] <= o->class_sites[k - 1])
      return fail(PT_EINVAL, "class_sites must ascend: [%u] = %u after %u", k, o->class_sites[k],
                  o->class_sites[k - 1]);
  }
  return PT_OK;
}

// Tile rows for a tiled-lane lattice: the tallest power of two up to 256 rows
// whose tile with halos for K sweeps fits the LDS budget (0 if none does).
uint32_t tile_rows(const Geometry &g, uint32_t K) {
  if (g.dim != 2 || g.plane % 32u || 2u * K > g.L / 2u) return 0;
  for (uint32_t H = std::min<uint32_t>(256u, g.L / 2u); H >= 8u; H /= 2u)
    if (tiled_lds_bytes(g, H, 2u * K) <= kTiledLds) return H;
  return 0;
}

}  // namespace

struct pt_server {
  pt_server_opts o{};
  uint8_t *base = nullptr;
  Head head{};
  BatchInst *d_insts = nullptr;
  uint32_t *d_ctr = nullptr;
  uint8_t *arena_base = nullptr;
  Arena arena;
  std::vector<Lane> lanes; // [0] batched, [1 .. tiled_lanes] tiled, then a batched lane per size class
  hipStream_t copy = nullptr;
  std::vector<hipEvent_t> event_pool;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> inst_job; // instance slot -> job id (0 = free)
  std::vector<uint32_t> free_inst;
  uint64_t resident = 0;
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

// Sweeps the device runs for a job in one cycle of K (at most K, never past
// its target or its next exchange point): the counters' rule, replayed.
uint64_t cycle_n(const Job &j, uint32_t K) {
  uint64_t n = std::min<uint64_t>(K, j.n_sweeps - j.queued);
  if (j.every) n = std::min<uint64_t>(n, j.every - j.queued % j.every);
  return n;
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
  std::vector<uint32_t> ctr(kCtrWords, 0u);
  j.wat.resize(R);
  j.att.resize(R);
  j.acc.resize(R);
  D2H(j.wat.data(), st.walker_at, R * 4);
  D2H(E.data(), st.E, R * 4);
  D2H(M.data(), st.M, R * 4);
  D2H(j.att.data(), st.att, R * 4);
  D2H(j.acc.data(), st.acc, R * 4);
  D2H(ctr.data(), sv->d_ctr + (size_t)j.inst * kCtrWords, kCtrWords * 4);
  j.n_records = records_between(c->cfg.record_every, 0, j.n_sweeps);
  j.Es.resize((size_t)j.n_records * R);
  j.Ms.resize((size_t)j.n_records * R);
  D2H(j.Es.data(), st.E_series, j.Es.size() * 4);
  D2H(j.Ms.data(), st.M_series, j.Ms.size() * 4);
  if (j.flags & PT_JOB_KEEP_SPINS) {
    j.bits.resize(R * N / 32);
    D2H(j.bits.data(), st.spins[j.cur], j.bits.size() * 4);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(sv->copy);
  if (e != hipSuccess) return e;
  j.sweeps_done = j.n_sweeps;
  j.exchanges_done = records_between(j.every, 0, j.n_sweeps);
  // the device's schedule must be the one the host replayed
  if (ctr[kCtrSweeps] != j.n_sweeps || ctr[kCtrExchanges] != j.exchanges_done ||
      ctr[kCtrRecords] != j.n_records || ctr[kCtrCur] != j.cur || ctr[kCtrActive] != 0u)
    return hipErrorUnknown;
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
  sv->inst_job[j.inst] = 0;
  sv->free_inst.push_back(j.inst);
  Lane &ln = sv->lanes[j.lane];
  ln.jobs.erase(std::find(ln.jobs.begin(), ln.jobs.end(), id));
  ln.slots -= (uint64_t)j.cfg.R * (j.tiles ? j.tiles : 1u);
  ln.work -= (uint64_t)j.cfg.R * j.sites();
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

// Admit queued jobs in arrival order while the head of the queue fits: an
// instance slot, its lane's walker (or walker-tile) slots and arena memory.
pt_status admit(pt_server *sv) {
  while (!sv->pending.empty()) {
    Job &j = *sv->jobs.at(sv->pending.front());
    if (sv->resident >= sv->o.max_jobs || sv->free_inst.empty()) break;
    uint32_t lane = 0;
    if (j.tiles) {
      // the tiled lane with the least resident work
      lane = 1;
      for (uint32_t l = 2; l <= sv->o.tiled_lanes; ++l)
        if (sv->lanes[l].work < sv->lanes[lane].work) lane = l;
    } else {
      // the batched lane of the smallest class that holds it (lane 0: above all classes)
      const uint32_t nc = n_classes(sv->o);
      for (uint32_t k = 0; k < nc && !lane; ++k)
        if (j.sites() <= sv->o.class_sites[k]) lane = sv->o.tiled_lanes + 1u + k;
    }
    Lane &ln = sv->lanes[lane];
    const uint64_t slots = (uint64_t)j.cfg.R * (j.tiles ? j.tiles : 1u);
    if (ln.slots + slots > sv->o.max_walkers) break;
    size_t off = 0;
    if (!sv->arena.alloc(j.bytes, &off)) break;
    sv->pending.pop_front();
    j.off = off;
    j.lane = lane;
    pt_status s = ctx_create(&j.cfg, ln.s, sv->arena_base + off, j.bytes, false, nullptr, &j.ctx);
    if (s != PT_OK) {
      sv->poisoned = true;
      return s;
    }
    j.admitted = now_s(sv->t0);
    ++sv->resident;
    j.inst = sv->free_inst.back();
    sv->free_inst.pop_back();
    sv->inst_job[j.inst] = j.id;
    ln.jobs.push_back(j.id);
    ln.slots += slots;
    ln.work += (uint64_t)j.cfg.R * j.sites();
    ln.dirty = true;
    // descriptor and counters, queued on the lane after its earlier work
    const BatchInst I = batch_inst(j.ctx, sv->d_ctr + (size_t)j.inst * kCtrWords);
    uint32_t ctr[kCtrWords] = {0u};
    ctr[kCtrTarget] = (uint32_t)j.n_sweeps;
    ctr[kCtrActive] = 1u;
    ctr[kCtrEvery] = j.every;
    ctr[kCtrCur] = 0u;
    ctr[kCtrTiles] = j.tiles;
    auto hi = bytes_of(&I, 1), hc = bytes_of(ctr, kCtrWords);
    hipError_t e = hipMemcpyAsync(sv->d_insts + j.inst, hi->data(), hi->size(), hipMemcpyHostToDevice, ln.s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(sv->d_ctr + (size_t)j.inst * kCtrWords, hc->data(), hc->size(),
                         hipMemcpyHostToDevice, ln.s);
    if (e != hipSuccess) return sv_fail(sv, e, "job admission");
    ln.staged.push_back(hi);
    ln.staged.push_back(hc);
  }
  return PT_OK;
}

// Rebuild a lane's work lists from its resident, unfinished jobs.
pt_status rebuild_lane(pt_server *sv, uint32_t l) {
  Lane &ln = sv->lanes[l];
  std::map<std::pair<uint32_t, uint32_t>, std::vector<uint64_t>> by_geo;
  std::vector<uint32_t> list;
  for (uint64_t id : ln.jobs) {
    Job &j = *sv->jobs.at(id);
    if (j.queued >= j.n_sweeps) continue;
    by_geo[{j.ctx->d.geo.dim, j.ctx->d.geo.L}].push_back(id);
    list.push_back(j.inst);
  }
  std::vector<BatchItem> items;
  std::vector<BatchTileItem> titems;
  std::vector<uint2> pairs;
  ln.groups.clear();
  for (auto &kv : by_geo) {
    Group G;
    G.g = sv->jobs.at(kv.second[0])->ctx->d.geo;
    for (uint64_t id : kv.second) G.max_R = std::max(G.max_R, sv->jobs.at(id)->cfg.R);
    if (!ln.tiled) {
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
    } else {
      const Job &j0 = *sv->jobs.at(kv.second[0]);
      G.H = G.g.L / j0.tiles;
      G.threads = G.H >= 256u ? 1024u : 512u;
      G.item_off = (uint32_t)titems.size();
      for (uint64_t id : kv.second) {
        const Job &j = *sv->jobs.at(id);
        for (uint32_t w = 0; w < j.cfg.R; ++w)
          for (uint32_t t = 0; t < j.tiles; ++t) titems.push_back({j.inst, w, t, 0u});
      }
      G.n_items = (uint32_t)titems.size() - G.item_off;
    }
    ln.groups.push_back(G);
  }
  // largest lattices first, so the longest workgroups start first
  std::sort(ln.groups.begin(), ln.groups.end(), [](const Group &x, const Group &y) {
    return x.g.N * (x.g.dim == 3 ? 4u : 1u) > y.g.N * (y.g.dim == 3 ? 4u : 1u);
  });
  ln.n_pairs = (uint32_t)pairs.size();
  ln.n_list = (uint32_t)list.size();
  hipError_t e = hipSuccess;
  auto up = [&](void *dst, auto &v) {
    if (e != hipSuccess || v.empty()) return;
    auto hv = bytes_of(v.data(), v.size());
    e = hipMemcpyAsync(dst, hv->data(), hv->size(), hipMemcpyHostToDevice, ln.s);
    ln.staged.push_back(hv);
  };
  up(ln.d_items, items);
  up(ln.d_titems, titems);
  up(ln.d_pairs, pairs);
  up(ln.d_list, list);
  if (e != hipSuccess) return sv_fail(sv, e, "lane work lists");
  ln.dirty = false;
  return PT_OK;
}

// Queue one cycle of lane l; *queued = false if it has nothing to run.
pt_status lane_cycle(pt_server *sv, uint32_t l, bool *queued) {
  *queued = false;
  Lane &ln = sv->lanes[l];
  if (ln.dirty) {
    pt_status s = rebuild_lane(sv, l);
    if (s != PT_OK) return s;
  }
  if (ln.groups.empty()) return PT_OK;
  const uint32_t K = ln.K;
  hipError_t e = hipSuccess;
  for (const Group &G : ln.groups) {
    if (e != hipSuccess) break;
    e = !ln.tiled ? launch_batch_sweep(sv->d_insts, ln.d_items + G.item_off, G.n_items, G.g, G.W,
                                       G.threads, K, ln.s)
                  : launch_batch_tiled(sv->d_insts, ln.d_titems + G.item_off, G.n_items, G.g, G.H,
                                       G.threads, K, ln.s);
  }
  if (e == hipSuccess && !ln.tiled && ln.n_pairs)
    e = launch_batch_exchange(sv->d_insts, ln.d_pairs, ln.n_pairs, K, ln.s);
  if (e == hipSuccess) e = launch_batch_advance(sv->d_insts, ln.d_list, ln.n_list, K, ln.s);
  if (e != hipSuccess) return sv_fail(sv, e, "lane cycle launch");
  Step st;
  // the device's schedule of this cycle, replayed on the host
  for (uint64_t id : ln.jobs) {
    Job &j = *sv->jobs.at(id);
    if (j.queued >= j.n_sweeps) continue;
    const uint64_t n = cycle_n(j, K);
    j.queued += n;
    if (n && j.tiles > 1u) j.cur ^= 1u;
    if (j.queued == j.n_sweeps) {
      st.finishing.push_back(id);
      ln.dirty = true;
    }
  }
  st.ev = take_event(sv);
  if (!st.ev) return sv_fail(sv, hipErrorOutOfMemory, "event creation");
  if ((e = hipEventRecord(st.ev, ln.s)) != hipSuccess) return sv_fail(sv, e, "step event");
  st.keep = std::move(ln.staged);
  ln.staged.clear();
  ln.q.push_back(std::move(st));
  if (ln.tiled) ++sv->tiled_steps;
  else ++sv->batched_cycles;
  *queued = true;
  return PT_OK;
}

pt_status top_up(pt_server *sv, bool *queued_any) {
  *queued_any = false;
  for (uint32_t l = 0; l < sv->lanes.size(); ++l) {
    while (sv->lanes[l].q.size() < sv->o.depth) {
      bool q = false;
      pt_status s = lane_cycle(sv, l, &q);
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
  sv->arena_base = sv->base + h.total;
  sv->arena.reset(ws_bytes - h.total, kAlign);
  sv->inst_job.assign(opts->max_jobs, 0);
  for (uint32_t i = opts->max_jobs; i-- > 0;) sv->free_inst.push_back(i);
  sv->lanes.resize(n_lanes(*opts));
  for (uint32_t l = 0; l < sv->lanes.size(); ++l) {
    Lane &ln = sv->lanes[l];
    ln.tiled = lane_tiled(*opts, l);
    if (!ln.tiled) {
      ln.d_items = (BatchItem *)(sv->base + h.items[l]);
      ln.d_pairs = (uint2 *)(sv->base + h.pairs[l]);
    } else {
      ln.d_titems = (BatchTileItem *)(sv->base + h.items[l]);
    }
    ln.d_list = (uint32_t *)(sv->base + h.list[l]);
    ln.K = ln.tiled ? opts->tiled_sweeps : opts->cycle_sweeps;
  }
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
  if ((cfg->L & (cfg->L - 1u)) || cfg->L < 8u)
    return fail(PT_EUNSUPPORTED, "served jobs need a power-of-two side of at least 8 (L = %u)", cfg->L);
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
  g.gpr = cfg->L / 8u;
  g.rows = dim == 3 ? cfg->L : 1u;
  g.plane = cfg->L * g.rows;
  g.nwr = (g.N + 31u) / 32u;
  g.phased = 0u;
  if (!batch_fits(g)) {
    // a tiled lane: tiles of H rows with halos for tiled_sweeps sweeps
    const uint32_t H = tile_rows(g, sv->o.tiled_sweeps);
    if (!H)
      return fail(PT_EUNSUPPORTED, "no tile of this lattice fits one workgroup's LDS with halos "
                  "for %u sweeps", sv->o.tiled_sweeps);
    j->tiles = g.L / H;
  }
  const uint64_t slots = (uint64_t)cfg->R * (j->tiles ? j->tiles : 1u);
  if (slots > sv->o.max_walkers)
    return fail(PT_ENOMEM, "job needs %llu walker slots, a lane holds %u", (unsigned long long)slots,
                sv->o.max_walkers);
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
  const size_t R = j.cfg.R, N = j.sites();
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
  out->walkers_resident = 0;
  for (const Lane &ln : sv->lanes) out->walkers_resident += ln.slots;
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
