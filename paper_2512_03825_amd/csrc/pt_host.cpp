// pt_host.cpp -- host side of the parallel-tempering Metropolis library: the C
// ABI of include/pt.h, configuration checks, the FP64 threshold tables, the
// workspace layout, plan selection and the launch schedule.
#include "pt_host.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <sys/stat.h>
#include <unistd.h>

using namespace ptmi;

namespace {
thread_local std::string g_err;
}  // namespace

namespace ptmi {

pt_status fail(pt_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

uint32_t records_between(uint32_t every, uint64_t s0, uint64_t s1) {
  return every ? (uint32_t)(s1 / every - s0 / every) : 0u;
}

uint32_t lg2(uint32_t v) {
  uint32_t r = 0;
  while ((1u << r) < v) ++r;
  return r;
}

}  // namespace ptmi

namespace {

bool is_pow2(uint32_t v) { return v && !(v & (v - 1u)); }

static_assert(kStaticScratchBytes == PT_STATIC_SCRATCH_BYTES, "scratch array size and its ABI constant differ");
static_assert(kMaxSweepsPerLaunch == PT_MAX_SWEEPS_PER_LAUNCH, "sweeps per launch and its ABI constant differ");

constexpr uint32_t kMaxR = 4096;
constexpr uint32_t kFusedChunk = 4096;   // sweeps per fused or persistent launch

// Saturation of the logistic swap rule: beyond |x| >= 32 ln 2 the decision no
// longer depends on the 32-bit draw.
constexpr double kSwapSat = 0x1.62e42fefa39efp+4;


// ---- acceptance rules, FP64, evaluated once per table entry ---------------
// Eq. (1) with the Boltzmann target of Eq. (2): accept a flip with energy
// change dE iff r < min(1, exp(-beta dE)) * 2^32; stored as the largest
// accepted r.  The caller guarantees p > 0.
uint32_t flip_threshold(double beta, double dE) {
  const double p = (dE <= 0.0) ? 1.0 : std::exp(-(beta * dE));
  const double q = std::ceil(std::ldexp(p, 32));
  const uint64_t n = std::min<uint64_t>((uint64_t)q, 1ull << 32); // accepted draws
  return (uint32_t)(n - 1u);
}

// Swap probability of Sec. 3, e^x/(1+e^x) evaluated as 1/(1+e^-x), x = dBeta * dE;
// returned as the number of accepted 32-bit draws (accept iff r < T).
uint64_t swap_threshold(double dbeta, double dE) {
  const double x = dbeta * dE;
  if (x >= kSwapSat) return 1ull << 32;
  if (x <= -kSwapSat) return 0;
  const double p = 1.0 / (1.0 + std::exp(-x));
  return (uint64_t)std::ceil(std::ldexp(p, 32));
}




pt_status derive(const pt_config *cfg, Derived *d) {
  if (!cfg) return fail(PT_EINVAL, "config is NULL");
  if (cfg->abi_version != PT_ABI_VERSION)
    return fail(PT_EINVAL, "abi_version %u, library expects %u", cfg->abi_version, PT_ABI_VERSION);
  if (cfg->model != PT_ISING2D && cfg->model != PT_EA3D)
    return fail(PT_EINVAL, "unknown model %u", cfg->model);
  const uint32_t dim = cfg->model == PT_EA3D ? 3u : 2u;
  const uint32_t maxL = dim == 3 ? 64u : 16384u;
  // the checkerboard needs an even side (periodic, two colours)
  if (cfg->L < 4u || (cfg->L & 1u) || cfg->L > maxL)
    return fail(PT_EINVAL, "L = %u: must be even, in [4, %u]", cfg->L, maxL);
  const bool phased = !is_pow2(cfg->L) || cfg->L < 8u;
  if (phased && dim == 3)
    return fail(PT_EUNSUPPORTED, "L = %u: the 3D kernels need a power of two in [8, 64]", cfg->L);
  if (cfg->R < 1u || cfg->R > kMaxR) return fail(PT_EINVAL, "R = %u: must be in [1, %u]", cfg->R, kMaxR);
  if (!cfg->beta) return fail(PT_EINVAL, "beta is NULL");
  if (dim == 2 && !std::isfinite(cfg->J)) return fail(PT_EINVAL, "J is not finite");
  if (!std::isfinite(cfg->h)) return fail(PT_EINVAL, "h is not finite");
  d->z = 2u * dim;
  d->jscale = dim == 2 ? cfg->J : 1.0;
  const double dEmax = 2.0 * (std::fabs(d->jscale) * d->z + (dim == 2 ? std::fabs(cfg->h) : 0.0));
  for (uint32_t k = 0; k < cfg->R; ++k) {
    const double b = cfg->beta[k];
    if (!std::isfinite(b) || b < 0.0) return fail(PT_EINVAL, "beta[%u] = %g: must be finite and >= 0", k, b);
    if (b * dEmax >= 700.0)
      return fail(PT_EINVAL, "beta[%u] * max dE = %g: flip probabilities would underflow", k, b * dEmax);
  }
  Geometry &g = d->geo;
  g.dim = dim;
  g.L = cfg->L;
  g.R = cfg->R;
  g.N = cfg->L * cfg->L * (dim == 3 ? cfg->L : 1u);
  g.gpr = cfg->L / 8u;
  g.rows = dim == 3 ? cfg->L : 1u;
  g.plane = cfg->L * g.rows;
  g.nwr = (g.N + 31u) / 32u;
  g.phased = phased ? 1u : 0u;
  if (phased && phased_lds_bytes(g) > max_lds_bytes())
    return fail(PT_EUNSUPPORTED, "L = %u: a 2D side that is not a power of two runs whole replicas "
                "in LDS, which needs %zu bytes (at most %zu)", cfg->L, phased_lds_bytes(g),
                max_lds_bytes());
  return PT_OK;
}

// Half-width of pair k's swap table: beyond it |x| >= 32 ln 2 + 1 (saturated).
uint32_t swap_half_width(const pt_config *cfg, const Derived &d, uint32_t k) {
  const double scale = std::fabs(d.jscale * (cfg->beta[k] - cfg->beta[k + 1]));
  const double dmax = (double)d.z * d.geo.N / 4.0; // |E_a - E_b| / 4 never exceeds this
  if (scale == 0.0) return 0;
  const double D = std::ceil((kSwapSat + 1.0) / (4.0 * scale));
  return (uint32_t)std::min(D, std::ceil(dmax));
}

size_t swap_entries(const pt_config *cfg, const Derived &d) {
  size_t n = 0;
  for (uint32_t k = 0; k + 1 < cfg->R; ++k) n += 2u * (size_t)swap_half_width(cfg, d, k) + 1u;
  return n;
}

Layout layout(const pt_config *cfg, const Derived &d) {
  const Geometry &g = d.geo;
  const size_t R = g.R, N = g.N;
  Layout l;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  l.spins[0] = take(R * g.nwr * 4); // bit-packed, ceil(N/32) words per walker
  l.spins[1] = take(R * g.nwr * 4);
  l.bonds = take(g.dim == 3 ? 3 * N / 8 : 0);
  // +-1 bytes the host uploads at create (only when the config provides them)
  size_t stage = 0;
  if (cfg->init_spins) stage = std::max(stage, R * N);
  if (cfg->couplings && g.dim == 3) stage = std::max(stage, 3 * N);
  l.staging = take(stage);
  l.flip = take(R * kClasses * 4);
  l.flipc = take(R * kClasses * 8);
  l.swap_tab = take(std::max<size_t>(swap_entries(cfg, d), 1) * 8);
  l.swap_off = take(R * 4);
  l.swap_D = take(R * 4);
  l.swap_sat = take(R * 16);
  l.wat = take(R * 4);
  l.sof = take(R * 4);
  l.E = take(R * 4);
  l.M = take(R * 4);
  l.att = take(R * 4);
  l.acc = take(R * 4);
  l.Es = take((size_t)cfg->max_records * R * 4);
  l.Ms = take((size_t)cfg->max_records * R * 4);
  l.counter = take(16);
  l.field = take(R * kFieldDigits * 8);
  l.fsign = take(R * 4);
  l.scratch = o;
  l.acc3 = take(kMaxSweepsPerLaunch * R * 16);
  l.mailbox = take(8 * kMaxParts * R * 8);
  l.halo = take(split_halo_words(g) * 8);
  l.total = o;
  return l;
}

void build_tables(const pt_config *cfg, const Derived &d, Tables *t) {
  const uint32_t R = cfg->R, z = d.z;
  t->flip.assign((size_t)R * kClasses, 0u);
  for (uint32_t k = 0; k < R; ++k)
    for (uint32_t b = 0; b < 2; ++b)
      for (uint32_t u = 0; u <= z; ++u) {
        // class (b, u): spin s = +-1 with u unsatisfied bonds, so s * F = z - 2u
        const int s = b ? -1 : 1;
        const int F = s * ((int)z - 2 * (int)u);
        const double dE = (d.geo.dim == 2)
                              ? (2.0 * (double)s) * (cfg->J * (double)F + cfg->h)
                              : (2.0 * (double)s) * (double)F;
        t->flip[(size_t)k * kClasses + 8u * b + u] = flip_threshold(cfg->beta[k], dE);
      }
  t->flipc.resize(t->flip.size());
  for (size_t i = 0; i < t->flip.size(); ++i)
    t->flipc[i] = (0xFFFFFFFFull << 32) | (uint64_t)(~t->flip[i]);
  t->off.assign(R, 0u);
  t->D.assign(R, 0u);
  t->sat.assign(2 * (size_t)R, 0u);
  t->swap.clear();
  for (uint32_t k = 0; k + 1 < R; ++k) {
    const uint32_t D = swap_half_width(cfg, d, k);
    const double db = cfg->beta[k] - cfg->beta[k + 1];
    auto rule = [&](int64_t dd) { return swap_threshold(db, d.jscale * (double)(4 * dd)); };
    t->off[k] = (uint32_t)t->swap.size();
    t->D[k] = D;
    for (int64_t dd = -(int64_t)D; dd <= (int64_t)D; ++dd) t->swap.push_back(rule(dd));
    t->sat[2 * k] = rule(-(int64_t)D - 1);
    t->sat[2 * k + 1] = rule((int64_t)D + 1);
  }
  if (t->swap.empty()) t->swap.push_back(0);
  // Field factor of a swap (2D, h != 0): digit j of |dM|/2 passes with
  // probability exp(-2^(j+1) |dBeta h|); sign of (dBeta * -h) decides when it applies.
  t->field.assign((size_t)R * kFieldDigits, 1ull << 32);
  t->fsign.assign(R, 0);
  if (d.geo.dim == 2 && cfg->h != 0.0)
    for (uint32_t k = 0; k + 1 < R; ++k) {
      const double db = cfg->beta[k] - cfg->beta[k + 1];
      const double c = db * -cfg->h;
      t->fsign[k] = c > 0.0 ? 1 : (c < 0.0 ? -1 : 0);
      const double a = std::fabs(db * cfg->h);
      for (uint32_t j = 0; j < kFieldDigits; ++j) {
        const double p = std::exp(-(a * std::ldexp(2.0, (int)j)));
        t->field[(size_t)k * kFieldDigits + j] = (uint64_t)std::ceil(std::ldexp(p, 32));
      }
    }
}

}  // namespace


namespace {

pt_status device_fail(pt_ctx *c, hipError_t e, const char *what) {
  if (c) c->poisoned = true;
  return fail(PT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Workgroups per walker of a persistent plan: L / tile_planes (1 for 0 or L).
uint32_t persist_parts(const Geometry &g, const pt_plan &p) {
  if (p.mode != PT_PLAN_PERSISTENT || p.tile_planes == 0u || p.tile_planes >= g.L) return 1u;
  return g.L / p.tile_planes;
}

pt_status check_plan(const pt_ctx *c, const pt_plan &p) {
  const Geometry &g = c->d.geo;
  if (g.phased) {
    // rows that are not whole 8-site groups: the whole-replica tiled plan only
    if (p.mode != PT_PLAN_TILED || p.tile_planes < g.L)
      return fail(PT_EINVAL, "L = %u is not a power of two (or below 8): only the tiled plan with "
                  "whole replicas (tile_planes >= L) runs it", g.L);
    if (p.block_threads < 64 || p.block_threads > 1024 || p.block_threads % 64)
      return fail(PT_EINVAL, "block_threads = %u: must be a multiple of 64 in [64, 1024]", p.block_threads);
    if (p.sweeps_per_launch < 1 || p.sweeps_per_launch > kMaxSweepsPerLaunch)
      return fail(PT_EINVAL, "sweeps_per_launch = %u: must be in [1, %u]", p.sweeps_per_launch,
                  kMaxSweepsPerLaunch);
    return PT_OK;
  }
  if (p.mode == PT_PLAN_LANES) { // block size follows R
    if (g.dim != 2 || (g.L != 8 && g.L != 16))
      return fail(PT_EINVAL, "the lanes plan holds a lattice in registers: 2D with L = 8 or 16 only");
    if (g.R > 1024) return fail(PT_EINVAL, "the lanes plan runs one workgroup: R <= 1024");
    if (lanes_lds_bytes(g) > max_lds_bytes())
      return fail(PT_EINVAL, "lanes plan needs %zu bytes of LDS (max %zu)", lanes_lds_bytes(g),
                  max_lds_bytes());
    return PT_OK;
  }
  if (p.mode == PT_PLAN_WAVE) { // block size follows R
    if (g.dim != 2 || (g.L != 8 && g.L != 16))
      return fail(PT_EINVAL, "the wave plan holds a lattice in one wavefront: 2D with L = 8 or 16 only");
    if (wave_threads(g) > 1024)
      return fail(PT_EINVAL, "the wave plan runs one workgroup: R L^2/8 = %u lanes exceed 1024",
                  g.R * (g.N / 8u));
    if (wave_lds_bytes(g) > max_lds_bytes())
      return fail(PT_EINVAL, "wave plan needs %zu bytes of LDS (max %zu)", wave_lds_bytes(g),
                  max_lds_bytes());
    return PT_OK;
  }
  if (p.block_threads < 64 || p.block_threads > 1024 || p.block_threads % 64)
    return fail(PT_EINVAL, "block_threads = %u: must be a multiple of 64 in [64, 1024]", p.block_threads);
  if (p.mode == PT_PLAN_FUSED) {
    if (fused_lds_bytes(g) > max_lds_bytes())
      return fail(PT_EINVAL, "fused plan needs %zu bytes of LDS (max %zu)", fused_lds_bytes(g),
                  max_lds_bytes());
    return PT_OK;
  }
  if (p.mode == PT_PLAN_PERSISTENT) {
    const uint32_t parts = persist_parts(g, p);
    if (parts > 1u && (g.L % p.tile_planes || (parts & (parts - 1u)) ||
                       parts > split_max_parts(g) || p.tile_planes < 8u))
      return fail(PT_EINVAL, "persistent plan: tile_planes = %u must be L (one workgroup per walker) "
                  "or L/P planes for P workgroups per walker (3D 16 <= L <= 32: P = 2; 2D 64 <= L <= "
                  "1024: P = 2, 4 or 8; at least 8 planes each)", p.tile_planes);
    const size_t lds = persist_lds_bytes(g, parts);
    if (lds > max_lds_bytes())
      return fail(PT_EINVAL, "persistent plan needs %zu bytes of LDS per workgroup (max %zu)", lds,
                  max_lds_bytes());
    const uint32_t cap = persist_max_workgroups(g, p.block_threads, parts);
    if (cap < parts * g.R)
      return fail(PT_EINVAL, "persistent plan needs %u co-resident workgroups, the device holds %u",
                  parts * g.R, cap);
    return PT_OK;
  }
  if (p.mode != PT_PLAN_TILED) return fail(PT_EINVAL, "unknown plan mode %u", p.mode);
  if (p.tile_planes < 1) return fail(PT_EINVAL, "tile_planes must be >= 1");
  if (p.sweeps_per_launch < 1 || p.sweeps_per_launch > kMaxSweepsPerLaunch)
    return fail(PT_EINVAL, "sweeps_per_launch = %u: must be in [1, %u]", p.sweeps_per_launch,
                kMaxSweepsPerLaunch);
  const uint32_t H = std::min(p.tile_planes, g.L);
  const uint32_t halo = H >= g.L ? 0u : 2u * p.sweeps_per_launch;
  if (halo && g.plane % 32u)
    return fail(PT_EINVAL, "tiles smaller than the lattice need planes of a multiple of 32 sites "
                "(2D: L >= 32)");
  if (halo > g.L / 2)
    return fail(PT_EINVAL, "halo of %u planes (2 per sweep per launch) exceeds L/2", halo);
  const size_t lds = tiled_lds_bytes(g, H, halo);
  if (lds > max_lds_bytes())
    return fail(PT_EINVAL, "tiled plan needs %zu bytes of LDS (max %zu)", lds, max_lds_bytes());
  return PT_OK;
}

pt_plan auto_plan(const pt_ctx *c) {
  const Geometry &g = c->d.geo;
  pt_plan p{};
  if (g.phased) {
    // whole replicas in place, the most sweeps per launch; with walkers for
    // every slot, workgroups of a whole number of waves per SIMD (a multiple
    // of 256 threads), as many as the workgroups that LDS lets share a compute
    // unit can hold together (2048 threads): 300^2 x 1500, three workgroups per
    // compute unit, measured 1.56e12 attempts/s at 512 threads against 1.22e12
    // at 320 and 1.16e12 at 384
    p.mode = PT_PLAN_TILED;
    p.tile_planes = g.L;
    p.sweeps_per_launch = kMaxSweepsPerLaunch;
    const uint32_t per_cu = (uint32_t)std::min<size_t>(4u, std::max<size_t>(1u, max_lds_bytes() / phased_lds_bytes(g)));
    p.block_threads = g.R >= 256u * per_cu ? std::min<uint32_t>(1024u, std::max<uint32_t>(256u, (2048u / per_cu) & ~255u))
                                           : 256u;
    return p;
  }
  // Small 2D lattices whose walkers fit one workgroup's wavefronts: no barrier
  // within a sweep (measured 1.1-1.8x the fused plan at L = 8 and 16).
  {
    pt_plan q{};
    q.mode = PT_PLAN_WAVE;
    q.block_threads = g.dim == 2 ? wave_threads(g) : 0u;
    q.tile_planes = g.L;
    q.sweeps_per_launch = 1;
    if (check_plan(c, q) == PT_OK) return q;
  }
  const size_t fused = fused_lds_bytes(g);
  const size_t work = (size_t)g.R * g.N * (g.dim == 3 ? 4u : 1u); // one workgroup's sites (EA: x4)
  if (fused <= 64u * 1024u && work <= 60u * 1024u) {
    // Small enough that one workgroup is the fastest: sweeps and exchanges
    // never leave the kernel.
    const uint32_t items = (g.R * g.N) / (8u * span_groups(g));
    p.mode = PT_PLAN_FUSED;
    p.block_threads = std::min<uint32_t>(1024u, std::max<uint32_t>(64u, (items + 63u) & ~63u));
    p.tile_planes = g.L;
    p.sweeps_per_launch = 1;
    return p;
  }
  // 3D walkers whose halves fit a workgroup's LDS, and enough compute units
  // for two workgroups per walker: each walker split over two co-resident
  // workgroups for a whole run, exchanges decided pairwise.
  if (g.dim == 3 && g.R >= 64) {
    pt_plan q{};
    q.mode = PT_PLAN_PERSISTENT;
    q.block_threads = 512; // 4 groups per item at L = 32 (measured best against 768, 1024)
    q.tile_planes = g.L / 2u;
    q.sweeps_per_launch = 1;
    if (check_plan(c, q) == PT_OK) return q;
  }
  // 2D walkers (h = 0) whose rows split over P co-resident workgroups of L/P
  // rows, with P R filling the device (one workgroup per compute unit): every
  // part stays in LDS for a whole run and trades two boundary rows per side
  // once per sweep (no launch, restaging or recomputed halo between sweeps).
  if (g.dim == 2 && split_max_parts(g)) {
    for (uint32_t P = 2u; P <= split_max_parts(g); P *= 2u) {
      if (persist_lds_bytes(g, P) > max_lds_bytes()) continue;
      pt_plan q{};
      q.mode = PT_PLAN_PERSISTENT;
      q.block_threads = 1024;
      q.tile_planes = g.L / P;
      q.sweeps_per_launch = 1;
      const uint32_t cap = persist_max_workgroups(g, q.block_threads, P);
      if (P * g.R > cap) break;                      // more parts only need more
      if (8u * P * g.R < 7u * cap) continue;        // most compute units idle: more parts
      if (check_plan(c, q) == PT_OK) return q;
      break;
    }
  }
  // Many walkers whose lattices fit a workgroup's LDS: one co-resident workgroup
  // per walker for a whole run, exchanges decided pairwise (no launch per sweep).
  if (g.R >= 128) {
    pt_plan q{};
    q.mode = PT_PLAN_PERSISTENT;
    q.block_threads = 1024;
    q.tile_planes = g.L;
    q.sweeps_per_launch = 1;
    if (check_plan(c, q) == PT_OK) return q;
  }
  p.mode = PT_PLAN_TILED;
  p.block_threads = 512;
  p.sweeps_per_launch = 2;
  if (g.dim == 3) {
    p.tile_planes = std::max<uint32_t>(g.L / 2u, 4u);
    p.sweeps_per_launch = 1;
    p.block_threads = 256;
  } else if (g.plane % 32u) {
    p.tile_planes = g.L; // small rows: whole-replica tiles, updated in place
    p.block_threads = 256;
  } else {
    // Tiles of full rows at four bits per site: the tallest tile (fewest
    // recomputed halo rows) that fits 144 KB of LDS with halos for 5 sweeps
    // per launch while the grid still gives every compute unit a workgroup.
    p.sweeps_per_launch = 5;
    uint32_t H = g.L;
    auto fits = [&](uint32_t h) {
      const uint32_t halo = h >= g.L ? 0u : 2u * p.sweeps_per_launch;
      return tiled_lds_bytes(g, h, halo) <= 144u * 1024u && (g.L / h) * g.R >= 256u;
    };
    while (H > 32u && !fits(H)) H /= 2u;
    p.tile_planes = H;
    p.block_threads = H >= 256u ? 1024u : 512u;
    if (H >= g.L) {
      // Whole replicas: no halo rows to recompute, so the most sweeps per
      // launch; when there are walkers for every slot, workgroups sized so that
      // the ones LDS lets share a compute unit hold 16 waves together
      // (measured: 256^2 x 1500 at 256 threads, 512^2 x 1500 at 1024).
      p.sweeps_per_launch = kMaxSweepsPerLaunch;
      const size_t lds = tiled_lds_bytes(g, H, 0u);
      const uint32_t per_cu = (uint32_t)std::min<size_t>(4u, std::max<size_t>(1u, max_lds_bytes() / lds));
      if (g.R >= 256u * per_cu) p.block_threads = 1024u / per_cu;
    }
  }
  for (int tries = 0; tries < 8 && check_plan(c, p) != PT_OK; ++tries) {
    // shrink until the plan fits (LDS, halo rules); whole-replica tiles always fit
    if (p.sweeps_per_launch > 1) p.sweeps_per_launch /= 2;
    else if (p.tile_planes > 1u && g.plane % 32u == 0) p.tile_planes /= 2;
    else p.tile_planes = g.L;
  }
  return p;
}

pt_status usable(pt_ctx *c) {
  if (!c) return fail(PT_EINVAL, "context is NULL");
  if (c->poisoned) return fail(PT_ESTATE, "context is poisoned by an earlier device error");
  return PT_OK;
}

// Threshold tables depend only on the model, the lattice size, the ladder, J
// and h; contexts with equal inputs (served jobs drawn from a few ladders) share
// one immutable copy instead of rebuilding it (up to ~10^6 exp() calls).
std::shared_ptr<const Tables> shared_tables(const pt_config *cfg, const Derived &d) {
  static std::mutex mu;
  static std::map<std::string, std::shared_ptr<const Tables>> cache;
  static std::vector<std::string> order; // insertion order, oldest first
  constexpr size_t kMaxCached = 256;
  std::string key;
  key.reserve(40 + 8 * (size_t)cfg->R);
  auto put = [&](const void *p, size_t n) { key.append(reinterpret_cast<const char *>(p), n); };
  put(&cfg->model, sizeof cfg->model);
  put(&d.geo.L, sizeof d.geo.L);
  put(&cfg->R, sizeof cfg->R);
  put(&cfg->J, sizeof cfg->J);
  put(&cfg->h, sizeof cfg->h);
  put(cfg->beta, (size_t)cfg->R * sizeof(double));
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  auto t = std::make_shared<Tables>();
  build_tables(cfg, d, t.get());
  std::lock_guard<std::mutex> lk(mu);
  auto ins = cache.emplace(key, t);
  if (ins.second) {
    order.push_back(key);
    if (order.size() > kMaxCached) {
      cache.erase(order.front());
      order.erase(order.begin());
    }
  }
  return ins.first->second;
}

}  // namespace

namespace ptmi {

pt_status ctx_advance(pt_ctx *c, uint32_t n, uint32_t every) {
  const uint32_t re = c->cfg.record_every;
  const uint32_t need = records_between(re, c->sweeps, c->sweeps + n);
  if ((uint64_t)c->n_records + need > c->cfg.max_records)
    return fail(PT_EINVAL, "%u more records would exceed max_records = %u", need, c->cfg.max_records);
  if (c->sweeps + n > 0xFFFFFFFFull) return fail(PT_EINVAL, "sweep counter would exceed 2^32");
  const Geometry &g = c->d.geo;
  if (c->static_scratch && n) {
    // the fixed array is shared by every such context on this device: tallies
    // must start at zero, and no post or mailbox word of another context may
    // carry a tag this run waits for
    const hipError_t err = launch_zero(c->static_scratch, c->lay.total - c->lay.scratch, c->stream);
    if (err != hipSuccess) return device_fail(c, err, "scratch clear");
  }
  uint32_t left = n;
  while (left) {
    Schedule sch{};
    sch.s0 = (uint32_t)c->sweeps;
    sch.record_every = re;
    sch.rec_base = c->n_records;
    sch.ex_step = (uint32_t)c->exchanges;
    uint32_t nsw, nex = 0;
    hipError_t err;
    if (c->plan.mode == PT_PLAN_FUSED || c->plan.mode == PT_PLAN_PERSISTENT ||
        c->plan.mode == PT_PLAN_LANES || c->plan.mode == PT_PLAN_WAVE) {
      nsw = std::min(left, kFusedChunk);
      sch.nsw = nsw;
      sch.exchange_every = every;
      nex = records_between(every, c->sweeps, c->sweeps + nsw);
      err = c->plan.mode == PT_PLAN_FUSED
                ? launch_fused(c->st, g, c->keys, c->cur, c->plan.block_threads, sch, c->stream)
            : c->plan.mode == PT_PLAN_LANES
                ? launch_lanes(c->st, g, c->keys, c->cur, sch, c->stream)
            : c->plan.mode == PT_PLAN_WAVE
                ? launch_wave(c->st, g, c->keys, c->cur, sch, c->stream)
                : launch_persist(c->st, g, c->keys, c->cur, c->plan.block_threads,
                                 persist_parts(g, c->plan), sch, c->wait_limit, c->stream);
    } else {
      nsw = std::min(left, c->plan.sweeps_per_launch);
      if (every) nsw = std::min<uint32_t>(nsw, every - (uint32_t)(c->sweeps % every));
      sch.nsw = nsw;
      sch.do_exchange = (every && (c->sweeps + nsw) % every == 0) ? 1u : 0u;
      nex = sch.do_exchange;
      const uint32_t H = std::min(c->plan.tile_planes, g.L);
      const uint32_t halo = H >= g.L ? 0u : 2u * nsw;
      err = launch_tiled(c->st, g, c->keys, c->cur, H, halo, c->plan.block_threads, sch, c->stream);
      if (err == hipSuccess && halo) c->cur ^= 1u;
    }
    if (err != hipSuccess) return device_fail(c, err, "sweep launch");
    c->n_records += records_between(re, c->sweeps, c->sweeps + nsw);
    c->sweeps += nsw;
    c->exchanges += nex;
    left -= nsw;
  }
  return PT_OK;
}

}  // namespace ptmi

pt_status ptmi::ctx_create(const pt_config *cfg, hipStream_t hip_stream, void *d_workspace,
                           size_t ws_bytes, bool sync, uint8_t *static_scratch, pt_ctx **out) {
  if (!out) return fail(PT_EINVAL, "out is NULL");
  *out = nullptr;
  Derived d;
  pt_status s = derive(cfg, &d);
  if (s != PT_OK) return s;
  if (cfg->record_every && cfg->max_records == 0)
    return fail(PT_EINVAL, "record_every > 0 needs max_records > 0");
  const size_t N = d.geo.N, R = d.geo.R;
  if (cfg->init_spins)
    for (size_t i = 0; i < R * N; ++i)
      if (cfg->init_spins[i] != 1 && cfg->init_spins[i] != -1)
        return fail(PT_EINVAL, "init_spins[%zu] = %d: must be +1 or -1", i, cfg->init_spins[i]);
  if (cfg->couplings && d.geo.dim == 3)
    for (size_t i = 0; i < 3 * N; ++i)
      if (cfg->couplings[i] != 1 && cfg->couplings[i] != -1)
        return fail(PT_EINVAL, "couplings[%zu] = %d: must be +1 or -1", i, cfg->couplings[i]);
  if (!d_workspace) return fail(PT_EINVAL, "workspace is NULL");
  if ((uintptr_t)d_workspace % kAlign) return fail(PT_EINVAL, "workspace must be 256-byte aligned");

  pt_ctx *c = new (std::nothrow) pt_ctx();
  if (!c) return fail(PT_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  c->beta.assign(cfg->beta, cfg->beta + cfg->R);
  c->cfg.beta = c->beta.data();
  c->cfg.init_spins = nullptr;
  c->cfg.couplings = nullptr;
  c->d = d;
  c->keys = {cfg->seed, cfg->stream_id, cfg->coupling_seed};
  // Laid out from the caller's config: its upload pointers size the staging area.
  c->lay = layout(cfg, d);
  const size_t need = static_scratch ? c->lay.scratch : c->lay.total;
  if (ws_bytes < need) {
    delete c;
    return fail(PT_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  }
  if (static_scratch && c->lay.total - c->lay.scratch > kStaticScratchBytes) {
    const size_t sb = c->lay.total - c->lay.scratch;
    delete c;
    return fail(PT_ENOMEM, "this configuration needs %zu bytes of scratch, the fixed array holds %zu",
                sb, kStaticScratchBytes);
  }
  c->static_scratch = static_scratch;
  c->tab = shared_tables(&c->cfg, d);
  c->stream = hip_stream;

  uint8_t *base = (uint8_t *)d_workspace;
  // scratch regions: in the workspace, or at the same offsets from the start
  // of the fixed array
  uint8_t *sbase = static_scratch ? static_scratch - c->lay.scratch : base;
  const Layout &l = c->lay;
  DevState &st = c->st;
  st.spins[0] = (uint32_t *)(base + l.spins[0]);
  st.spins[1] = (uint32_t *)(base + l.spins[1]);
  st.bonds = (uint32_t *)(base + l.bonds);
  st.flip_thr = (uint32_t *)(base + l.flip);
  st.flip_cmp = (uint64_t *)(base + l.flipc);
  st.swap_tab = (uint64_t *)(base + l.swap_tab);
  st.swap_off = (uint32_t *)(base + l.swap_off);
  st.swap_D = (uint32_t *)(base + l.swap_D);
  st.swap_sat = (uint64_t *)(base + l.swap_sat);
  st.swap_n = (uint32_t)c->tab->swap.size();
  st.field_thr = (uint64_t *)(base + l.field);
  st.field_sign = (int32_t *)(base + l.fsign);
  st.walker_at = (uint32_t *)(base + l.wat);
  st.slot_of = (uint32_t *)(base + l.sof);
  st.E = (int32_t *)(base + l.E);
  st.M = (int32_t *)(base + l.M);
  st.acc3 = (int32_t *)(sbase + l.acc3);
  st.att = (uint32_t *)(base + l.att);
  st.acc = (uint32_t *)(base + l.acc);
  st.E_series = (int32_t *)(base + l.Es);
  st.M_series = (int32_t *)(base + l.Ms);
  st.counter = (uint32_t *)(base + l.counter);
  st.mailbox = (uint64_t *)(sbase + l.mailbox);
  st.halo = (uint64_t *)(sbase + l.halo);
  st.staging = base + l.staging;

  hipError_t e = hipSuccess;
  const hipStream_t sm = c->stream;
  auto H2D = [&](void *dst, const void *src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, sm);
  };
  H2D(st.flip_thr, c->tab->flip.data(), c->tab->flip.size() * 4);
  H2D(st.flip_cmp, c->tab->flipc.data(), c->tab->flipc.size() * 8);
  H2D(st.swap_tab, c->tab->swap.data(), c->tab->swap.size() * 8);
  H2D(st.swap_off, c->tab->off.data(), R * 4);
  H2D(st.swap_D, c->tab->D.data(), R * 4);
  H2D(st.swap_sat, c->tab->sat.data(), R * 16);
  H2D(st.field_thr, c->tab->field.data(), c->tab->field.size() * 8);
  H2D(st.field_sign, c->tab->fsign.data(), R * 4);
  if (e == hipSuccess) e = launch_reset(st, d.geo, sm);
  if (d.geo.dim == 3) {
    if (cfg->couplings) H2D(st.staging, cfg->couplings, 3 * N);
    if (e == hipSuccess) e = launch_init_bonds(st, d.geo, c->keys, cfg->couplings != nullptr, sm);
  }
  if (cfg->init_spins) H2D(st.staging, cfg->init_spins, R * N);
  if (e == hipSuccess) e = launch_init_spins(st, d.geo, c->keys, cfg->init_spins != nullptr, sm);
  if (e == hipSuccess) e = launch_recount(st, d.geo, 0, sm);
  if (e == hipSuccess && sync) e = hipStreamSynchronize(sm);
  if (e != hipSuccess) {
    delete c;
    return fail(PT_EDEVICE, "initialisation: %s", hipGetErrorString(e));
  }
  c->plan = auto_plan(c);
  *out = c;
  return PT_OK;
}

extern "C" {

size_t pt_workspace_bytes(const pt_config *cfg) {
  Derived d;
  if (derive(cfg, &d) != PT_OK) return 0;
  return layout(cfg, d).total;
}

pt_status pt_create(const pt_config *cfg, void *hip_stream, void *d_workspace, size_t ws_bytes,
                    pt_ctx **out) {
  return ctx_create(cfg, (hipStream_t)hip_stream, d_workspace, ws_bytes, true, nullptr, out);
}

pt_status pt_create_static(const pt_config *cfg, void *hip_stream, void *d_state,
                           size_t *state_bytes, pt_ctx **out) {
  if (out) *out = nullptr;
  if (!state_bytes) return fail(PT_EINVAL, "state_bytes is NULL");
  Derived d;
  pt_status s = derive(cfg, &d);
  if (s != PT_OK) return s;
  const Layout l = layout(cfg, d);
  if (l.total - l.scratch > kStaticScratchBytes)
    return fail(PT_ENOMEM, "this configuration needs %zu bytes of scratch, the fixed array holds %zu",
                l.total - l.scratch, kStaticScratchBytes);
  if (!d_state) { // size query
    *state_bytes = l.scratch;
    return PT_OK;
  }
  if ((uintptr_t)d_state % kAlign) return fail(PT_EINVAL, "workspace must be 256-byte aligned");
  if (*state_bytes < l.scratch)
    return fail(PT_ENOMEM, "workspace of %zu bytes, need %zu", *state_bytes, l.scratch);
  uint8_t *scr = nullptr;
  const hipError_t e = static_scratch(&scr);
  if (e != hipSuccess) return fail(PT_EDEVICE, "scratch array address: %s", hipGetErrorString(e));
  return ctx_create(cfg, (hipStream_t)hip_stream, d_state, *state_bytes, true, scr, out);
}

pt_status pt_set_plan(pt_ctx *ctx, const pt_plan *plan) {
  pt_status s = usable(ctx);
  if (s != PT_OK) return s;
  if (!plan) return fail(PT_EINVAL, "plan is NULL");
  if (plan->mode == PT_PLAN_AUTO) {
    ctx->plan = auto_plan(ctx);
    return PT_OK;
  }
  s = check_plan(ctx, *plan);
  if (s != PT_OK) return s;
  ctx->plan = *plan;
  if (ctx->plan.mode == PT_PLAN_FUSED || ctx->plan.mode == PT_PLAN_PERSISTENT ||
      ctx->plan.mode == PT_PLAN_LANES || ctx->plan.mode == PT_PLAN_WAVE) {
    if (persist_parts(ctx->d.geo, ctx->plan) == 1u) ctx->plan.tile_planes = ctx->d.geo.L;
    ctx->plan.sweeps_per_launch = 1;
  }
  if (ctx->plan.mode == PT_PLAN_LANES) ctx->plan.block_threads = (ctx->d.geo.R + 63u) & ~63u;
  if (ctx->plan.mode == PT_PLAN_WAVE) ctx->plan.block_threads = wave_threads(ctx->d.geo);
  return PT_OK;
}

pt_status pt_get_plan(const pt_ctx *ctx, pt_plan *plan) {
  if (!ctx || !plan) return fail(PT_EINVAL, "NULL argument");
  *plan = ctx->plan;
  return PT_OK;
}

pt_status pt_set_wait_limit(pt_ctx *ctx, uint32_t polls) {
  pt_status s = usable(ctx);
  if (s != PT_OK) return s;
  ctx->wait_limit = polls;
  return PT_OK;
}

pt_status pt_sweep(pt_ctx *ctx, uint32_t n_sweeps) {
  pt_status s = usable(ctx);
  if (s != PT_OK) return s;
  return ctx_advance(ctx, n_sweeps, 0);
}

pt_status pt_exchange(pt_ctx *ctx) {
  pt_status s = usable(ctx);
  if (s != PT_OK) return s;
  hipError_t e = launch_exchange(ctx->st, ctx->d.geo, ctx->keys, (uint32_t)ctx->exchanges, ctx->stream);
  if (e != hipSuccess) return device_fail(ctx, e, "exchange launch");
  ctx->exchanges++;
  return PT_OK;
}

pt_status pt_run(pt_ctx *ctx, uint32_t n_sweeps, uint32_t exchange_every) {
  pt_status s = usable(ctx);
  if (s != PT_OK) return s;
  return ctx_advance(ctx, n_sweeps, exchange_every);
}

pt_status pt_observables(pt_ctx *ctx, pt_obs *obs) {
  pt_status s = usable(ctx);
  if (s != PT_OK) return s;
  if (!obs) return fail(PT_EINVAL, "obs is NULL");
  const size_t R = ctx->d.geo.R, N = ctx->d.geo.N;
  if (obs->spins && obs->spins_slot != PT_ALL_SLOTS && obs->spins_slot >= R)
    return fail(PT_EINVAL, "spins_slot = %u out of range", obs->spins_slot);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return device_fail(ctx, e, "stream synchronise");
  const DevState &st = ctx->st;
  std::vector<uint32_t> wat(R), att(R), acc(R);
  std::vector<int32_t> E(R), M(R);
  auto D2H = [&](void *dst, const void *src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpy(dst, src, n, hipMemcpyDeviceToHost);
  };
  D2H(wat.data(), st.walker_at, R * 4);
  D2H(E.data(), st.E, R * 4);
  D2H(M.data(), st.M, R * 4);
  D2H(att.data(), st.att, R * 4);
  D2H(acc.data(), st.acc, R * 4);
  uint32_t flags[4] = {0, 0, 0, 0};
  D2H(flags, st.counter, sizeof flags);
  if (obs->E_series) D2H(obs->E_series, st.E_series, (size_t)ctx->n_records * R * 4);
  if (obs->M_series) D2H(obs->M_series, st.M_series, (size_t)ctx->n_records * R * 4);
  std::vector<uint32_t> bits; // packed walker lattices
  const size_t wpr = ctx->d.geo.nwr;
  if (obs->spins) {
    if (obs->spins_slot == PT_ALL_SLOTS) {
      bits.resize(R * wpr);
      D2H(bits.data(), st.spins[ctx->cur], R * wpr * 4);
    } else {
      bits.resize(wpr);
      if (e == hipSuccess && wat[obs->spins_slot] < R)
        D2H(bits.data(), st.spins[ctx->cur] + (size_t)wat[obs->spins_slot] * wpr, wpr * 4);
    }
  }
  if (e != hipSuccess) return device_fail(ctx, e, "observables copy");
  if (flags[1]) {
    ctx->poisoned = true;
    return fail(PT_EDEVICE, "a persistent launch stopped: a pairwise exchange wait exceeded its bound");
  }
  for (size_t k = 0; k < R; ++k)
    if (wat[k] >= R) {
      ctx->poisoned = true;
      return fail(PT_EDEVICE, "walker map corrupted (slot %zu holds %u)", k, wat[k]);
    }
  if (obs->walker_at) std::memcpy(obs->walker_at, wat.data(), R * 4);
  for (size_t k = 0; k < R; ++k) {
    if (obs->E_slot) obs->E_slot[k] = E[wat[k]];
    if (obs->M_slot) obs->M_slot[k] = M[wat[k]];
  }
  if (obs->swap_att || obs->swap_acc) {
    if (obs->swap_att) std::memset(obs->swap_att, 0, R * R * 8);
    if (obs->swap_acc) std::memset(obs->swap_acc, 0, R * R * 8);
    for (size_t k = 0; k + 1 < R; ++k) {
      if (obs->swap_att) obs->swap_att[k * R + k + 1] = obs->swap_att[(k + 1) * R + k] = att[k];
      if (obs->swap_acc) obs->swap_acc[k * R + k + 1] = obs->swap_acc[(k + 1) * R + k] = acc[k];
    }
  }
  auto unpack = [&](const uint32_t *src, int8_t *dst) {
    for (size_t i = 0; i < N; ++i) dst[i] = ((src[i >> 5] >> (i & 31)) & 1u) ? -1 : 1;
  };
  if (obs->spins) {
    if (obs->spins_slot == PT_ALL_SLOTS) {
      for (size_t k = 0; k < R; ++k) unpack(bits.data() + (size_t)wat[k] * wpr, obs->spins + k * N);
    } else {
      unpack(bits.data(), obs->spins);
    }
  }
  obs->sweeps_done = ctx->sweeps;
  obs->exchanges_done = ctx->exchanges;
  obs->n_records = ctx->n_records;
  return PT_OK;
}

pt_status pt_flip_thresholds(const pt_ctx *ctx, uint32_t *out) {
  if (!ctx || !out) return fail(PT_EINVAL, "NULL argument");
  std::memcpy(out, ctx->tab->flip.data(), ctx->tab->flip.size() * 4);
  return PT_OK;
}

pt_status pt_swap_threshold(const pt_ctx *ctx, uint32_t k, int64_t d, uint64_t *out_T) {
  if (!ctx || !out_T) return fail(PT_EINVAL, "NULL argument");
  if (k + 1 >= ctx->d.geo.R) return fail(PT_EINVAL, "pair %u out of range", k);
  const int64_t D = ctx->tab->D[k];
  if (d < -D)
    *out_T = ctx->tab->sat[2 * (size_t)k];
  else if (d > D)
    *out_T = ctx->tab->sat[2 * (size_t)k + 1];
  else
    *out_T = ctx->tab->swap[ctx->tab->off[k] + (size_t)(d + D)];
  return PT_OK;
}

void pt_destroy(pt_ctx *ctx) { delete ctx; }

const char *pt_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---- batched form -------------------------------------------------------------
namespace {

struct BatchGroup {
  Geometry g;                 // dim, L (R varies inside the group)
  std::vector<uint32_t> inst; // instance indices
  uint32_t max_R = 0;
  uint32_t W = 1, threads = 256;
  uint32_t item_off = 0;      // into the device item array
  std::vector<BatchItem> items;
  // online tuning: candidate (W, threads) pairs timed on real cycles
  std::vector<std::pair<uint32_t, uint32_t>> cand;
  std::vector<float> cand_ms;
  bool tuned = false;
};

// Decompositions found fastest by the online tuner, keyed by what decides
// them -- the device (architecture and compute units), the model, the lattice
// side and the replica count rounded up to a power of two -- and kept in a
// text file so that later processes start tuned: $PTMI_TUNE_CACHE, else
// $XDG_CACHE_HOME/ptmi/batch_tuning.txt or ~/.cache/ptmi/batch_tuning.txt
// (PTMI_TUNE_CACHE set but empty: this process only).  One "key = value" line
// per entry; unreadable or malformed files are ignored, write failures too.
// The entries in memory follow the file: when the path changes (a process
// that sets PTMI_TUNE_CACHE anew) they are dropped and the new file is read.
// Decompositions never change results, so a stale entry only costs speed.
std::mutex g_tuned_mu;
std::map<std::string, std::string> g_tuned; // guarded by g_tuned_mu
bool g_tuned_loaded = false;
std::string g_tuned_path;

std::string tune_cache_path() {
  const char *p = std::getenv("PTMI_TUNE_CACHE");
  if (p) return p;
  const char *x = std::getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/ptmi/batch_tuning.txt";
  const char *h = std::getenv("HOME");
  if (h && *h) return std::string(h) + "/.cache/ptmi/batch_tuning.txt";
  return "";
}

// Called with g_tuned_mu held.
void tune_cache_load() {
  const std::string path = tune_cache_path();
  if (g_tuned_loaded && path == g_tuned_path) return;
  g_tuned_loaded = true;
  g_tuned_path = path;
  g_tuned.clear();
  if (path.empty()) return;
  FILE *f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    std::string l(line);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
    const size_t eq = l.find(" = ");
    if (eq == std::string::npos || eq == 0) continue;
    g_tuned[l.substr(0, eq)] = l.substr(eq + 3);
  }
  std::fclose(f);
}

// Called with g_tuned_mu held: record an entry and rewrite the file (written
// to a temporary name and renamed, so readers never see half a file).
void tune_cache_put(const std::string &key, const std::string &value) {
  g_tuned[key] = value;
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  for (size_t i = 1; i < path.size(); ++i) // create the directories on the way
    if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const auto &kv : g_tuned) std::fprintf(f, "%s = %s\n", kv.first.c_str(), kv.second.c_str());
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) (void)std::remove(tmp.c_str());
}

// The current device, as the cache keys name it.
std::string device_key() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string arch(prop.gcnArchName);
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

uint32_t pow2_at_least(uint32_t v) {
  uint32_t p = 1;
  while (p < v) p *= 2u;
  return p;
}

std::string group_key(const std::string &dev, const Geometry &g, uint32_t max_R) {
  char buf[160];
  std::snprintf(buf, sizeof buf, "group %s %s L=%u R<=%u", dev.c_str(), g.dim == 3 ? "ea3d" : "ising2d",
                g.L, pow2_at_least(max_R));
  return buf;
}

std::vector<std::pair<uint32_t, uint32_t>> batch_candidates(const Geometry &g, uint32_t max_R) {
  std::vector<std::pair<uint32_t, uint32_t>> c;
  const uint32_t spans = g.N / (8u * batch_span(g));
  for (uint32_t W = 1; W <= 32 && W <= max_R; W *= 2) {
    if (batch_lds_bytes(g, W) > 64u * 1024u) break;
    const uint32_t work = W * spans; // lanes' worth of work per half sweep
    uint32_t t = std::min<uint32_t>(512u, std::max<uint32_t>(64u, ((work / 2u) + 63u) & ~63u));
    c.push_back({W, t});
    if (t > 64u) c.push_back({W, t / 2u});
  }
  if (c.empty()) c.push_back({1u, 256u});
  return c;
}

}  // namespace

namespace ptmi {

BatchInst batch_inst(const pt_ctx *c, uint32_t *ctr) {
  const Geometry &g = c->d.geo;
  BatchInst I;
  I.st = c->st;
  I.geo = g;
  I.key = c->keys;
  I.record_every = c->cfg.record_every;
  const uint32_t V = batch_span(g);
  I.lg_L = lg2(g.L);
  I.lg_spr = lg2(g.gpr / V);
  I.lg_rows = lg2(g.rows);
  I.lg_items = lg2(g.N / (8u * V));
  I.z2 = g.dim == 3 ? 12 : 8;
  I.ctr = ctr;
  return I;
}

bool batch_fits(const Geometry &g) { return batch_lds_bytes(g, 1) <= max_lds_bytes(); }

std::pair<uint32_t, uint32_t> batch_decomposition(const Geometry &g, uint32_t max_R) {
  const std::string key = group_key(device_key(), g, max_R);
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    tune_cache_load();
    auto it = g_tuned.find(key);
    unsigned W = 0, T = 0;
    if (it != g_tuned.end() && std::sscanf(it->second.c_str(), "W=%u threads=%u", &W, &T) == 2 &&
        W >= 1 && T >= 64 && T <= 1024 && T % 64 == 0)
      return {std::min<uint32_t>(W, max_R), T};
  }
  return batch_candidates(g, max_R)[0];
}

}  // namespace ptmi

struct pt_batch {
  std::vector<pt_ctx *> ctx;
  hipStream_t user = nullptr, own = nullptr;
  hipEvent_t ev_sync = nullptr;
  std::vector<hipEvent_t> tune_ev; // [groups][2] start / end of a timed sweep launch
  BatchInst *d_insts = nullptr;
  BatchItem *d_items = nullptr;
  uint2 *d_pairs = nullptr;
  uint32_t *d_ctr = nullptr;
  uint32_t n_pairs = 0;
  std::vector<BatchGroup> groups;
  std::vector<uint2> pairs;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t graph_K = 0;
  bool graph_dirty = true;
  bool poisoned = false;
  std::string dev;       // device key of the tuning cache
  // sweeps per cycle: tuned per (device, mix of groups, exchange interval) over
  // the divisors of the interval up to 16, one timed cycle each
  uint32_t K = 0;        // the value of the last run
  std::map<uint32_t, uint32_t> K_best; // exchange interval -> tuned K
};

namespace {

struct BatchLayoutHost {
  std::vector<size_t> slice;
  size_t insts, ctr, items, pairs, total;
};

BatchLayoutHost batch_host_layout(const pt_config *cfgs, uint32_t n, pt_status *st) {
  BatchLayoutHost l;
  size_t o = 0, sumR = 0, sumP = 0;
  *st = PT_OK;
  for (uint32_t i = 0; i < n; ++i) {
    const size_t b = pt_workspace_bytes(&cfgs[i]);
    if (!b) {
      *st = PT_EINVAL;
      return l;
    }
    l.slice.push_back(o);
    o = align_up(o + b);
    sumR += cfgs[i].R;
    sumP += cfgs[i].R - 1;
  }
  l.insts = o;
  o = align_up(o + n * sizeof(BatchInst));
  l.ctr = o;
  o = align_up(o + n * kCtrWords * 4);
  l.items = o;
  o = align_up(o + sumR * sizeof(BatchItem));
  l.pairs = o;
  o = align_up(o + std::max<size_t>(sumP, 1) * sizeof(uint2));
  l.total = o;
  return l;
}

pt_status batch_fail(pt_batch *b, hipError_t e, const char *what) {
  if (b) b->poisoned = true;
  return fail(PT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void build_items(pt_batch *b, BatchGroup &G) {
  G.items.clear();
  for (uint32_t i : G.inst)
    for (uint32_t w0 = 0; w0 < b->ctx[i]->d.geo.R; w0 += G.W) G.items.push_back({i, w0});
}

hipError_t upload_items(pt_batch *b, BatchGroup &G, hipStream_t s) {
  return hipMemcpyAsync(b->d_items + G.item_off, G.items.data(), G.items.size() * sizeof(BatchItem),
                        hipMemcpyHostToDevice, s);
}

hipError_t launch_cycle(pt_batch *b, uint32_t K, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (auto &G : b->groups) {
    e = launch_batch_sweep(b->d_insts, b->d_items + G.item_off, (uint32_t)G.items.size(), G.g, G.W,
                           G.threads, K, s);
    if (e != hipSuccess) return e;
  }
  if ((e = launch_batch_exchange(b->d_insts, b->d_pairs, b->n_pairs, K, s)) != hipSuccess) return e;
  return launch_batch_advance(b->d_insts, nullptr, (uint32_t)b->ctx.size(), K, s);
}

}  // namespace

extern "C" {

size_t pt_batch_workspace_bytes(const pt_config *cfgs, uint32_t n) {
  if (!cfgs || n == 0) {
    fail(PT_EINVAL, "empty batch");
    return 0;
  }
  pt_status st;
  BatchLayoutHost l = batch_host_layout(cfgs, n, &st);
  return st == PT_OK ? l.total : 0;
}

pt_status pt_batch_create(const pt_config *cfgs, uint32_t n, void *hip_stream, void *d_workspace,
                          size_t ws_bytes, pt_batch **out) {
  if (!out) return fail(PT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfgs || n == 0) return fail(PT_EINVAL, "empty batch");
  pt_status st;
  BatchLayoutHost l = batch_host_layout(cfgs, n, &st);
  if (st != PT_OK) return st;
  for (uint32_t i = 0; i < n; ++i)
    if ((cfgs[i].L & (cfgs[i].L - 1u)) || cfgs[i].L < 8u)
      return fail(PT_EUNSUPPORTED, "instance %u: batched instances need a power-of-two side of at "
                  "least 8 (L = %u)", i, cfgs[i].L);
  if (!d_workspace || (uintptr_t)d_workspace % kAlign) return fail(PT_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < l.total) return fail(PT_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, l.total);
  pt_batch *b = new (std::nothrow) pt_batch();
  if (!b) return fail(PT_ENOMEM, "host allocation failed");
  b->user = (hipStream_t)hip_stream;
  uint8_t *base = (uint8_t *)d_workspace;
  for (uint32_t i = 0; i < n; ++i) {
    pt_ctx *c = nullptr;
    st = pt_create(&cfgs[i], hip_stream, base + l.slice[i], pt_workspace_bytes(&cfgs[i]), &c);
    if (st != PT_OK) {
      pt_batch_destroy(b);
      return st;
    }
    b->ctx.push_back(c);
  }
  b->d_insts = (BatchInst *)(base + l.insts);
  b->d_ctr = (uint32_t *)(base + l.ctr);
  b->d_items = (BatchItem *)(base + l.items);
  b->d_pairs = (uint2 *)(base + l.pairs);
  std::vector<BatchInst> hi(n);
  std::map<std::pair<uint32_t, uint32_t>, size_t> gidx;
  for (uint32_t i = 0; i < n; ++i) {
    const pt_ctx *c = b->ctx[i];
    const Geometry &g = c->d.geo;
    hi[i] = batch_inst(c, b->d_ctr + (size_t)i * kCtrWords);
    for (uint32_t k = 0; k + 1 < g.R; ++k) b->pairs.push_back(make_uint2(i, k));
    const auto key = std::make_pair(g.dim, g.L);
    if (!gidx.count(key)) {
      gidx[key] = b->groups.size();
      b->groups.emplace_back();
      b->groups.back().g = g;
    }
    BatchGroup &G = b->groups[gidx[key]];
    G.inst.push_back(i);
    G.max_R = std::max(G.max_R, g.R);
  }
  // largest lattices first, so the longest workgroups start first
  std::sort(b->groups.begin(), b->groups.end(),
            [](const BatchGroup &x, const BatchGroup &y) { return x.g.N * (x.g.dim == 3 ? 4 : 1) > y.g.N * (y.g.dim == 3 ? 4 : 1); });
  uint32_t off = 0;
  b->dev = device_key();
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    tune_cache_load();
    for (auto &G : b->groups) {
      G.cand = batch_candidates(G.g, G.max_R);
      G.W = G.cand[0].first;
      G.threads = G.cand[0].second;
      auto it = g_tuned.find(group_key(b->dev, G.g, G.max_R));
      unsigned W = 0, T = 0;
      if (it != g_tuned.end() && std::sscanf(it->second.c_str(), "W=%u threads=%u", &W, &T) == 2 &&
          W >= 1 && T >= 64 && T <= 1024 && T % 64 == 0 && batch_lds_bytes(G.g, W) <= max_lds_bytes()) {
        G.W = std::min<uint32_t>(W, G.max_R);
        G.threads = T;
        G.tuned = true;
      }
      G.item_off = off;
      uint32_t sumR = 0;
      for (uint32_t i : G.inst) sumR += b->ctx[i]->d.geo.R;
      off += sumR; // room for W = 1
      build_items(b, G);
    }
  }
  b->n_pairs = (uint32_t)b->pairs.size();
  std::vector<uint32_t> zeros((size_t)n * kCtrWords, 0u);
  hipError_t e = hipMemcpyAsync(b->d_insts, hi.data(), n * sizeof(BatchInst), hipMemcpyHostToDevice, b->user);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_ctr, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice, b->user);
  if (e == hipSuccess && b->n_pairs)
    e = hipMemcpyAsync(b->d_pairs, b->pairs.data(), b->pairs.size() * sizeof(uint2), hipMemcpyHostToDevice, b->user);
  for (auto &G : b->groups)
    if (e == hipSuccess) e = upload_items(b, G, b->user);
  if (e == hipSuccess) e = hipStreamSynchronize(b->user);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_sync, hipEventDisableTiming);
  b->tune_ev.assign(2 * b->groups.size(), nullptr);
  for (hipEvent_t &ev : b->tune_ev)
    if (e == hipSuccess) e = hipEventCreate(&ev);
  if (e != hipSuccess) {
    pt_batch_destroy(b);
    return fail(PT_EDEVICE, "batch initialisation: %s", hipGetErrorString(e));
  }
  *out = b;
  return PT_OK;
}

}  // extern "C"

namespace {

// Key of the sweeps-per-cycle choice: the device, the exchange interval and
// every lattice-size group of the batch.
std::string mix_key(const pt_batch *b, uint32_t every) {
  std::string k = "cycle " + b->dev + " every=" + std::to_string(every);
  for (const auto &G : b->groups)
    k += std::string(" ") + (G.g.dim == 3 ? "ea3d" : "ising2d") + ":" + std::to_string(G.g.L) + ":" +
         std::to_string(pow2_at_least(G.max_R));
  return k;
}

// (Re)capture one cycle of K sweeps in the batch's graph if needed.
hipError_t batch_graph(pt_batch *b, uint32_t K) {
  if (!b->graph_dirty && b->graph_K == K) return hipSuccess;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  hipError_t e = hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = launch_cycle(b, K, b->own);
    e = hipStreamEndCapture(b->own, &b->graph);
    if (e == hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e == hipSuccess) {
    b->graph_K = K;
    b->graph_dirty = false;
  }
  return e;
}

}  // namespace

extern "C" {

pt_status pt_batch_run(pt_batch *b, uint32_t n_sweeps, uint32_t exchange_every) {
  if (!b) return fail(PT_EINVAL, "batch is NULL");
  if (b->poisoned) return fail(PT_ESTATE, "batch is poisoned by an earlier device error");
  if (n_sweeps == 0) return PT_OK;
  for (pt_ctx *c : b->ctx) {
    const uint32_t need = records_between(c->cfg.record_every, c->sweeps, c->sweeps + n_sweeps);
    if ((uint64_t)c->n_records + need > c->cfg.max_records)
      return fail(PT_EINVAL, "%u more records would exceed max_records = %u", need, c->cfg.max_records);
    if (c->sweeps + n_sweeps > 0xFFFFFFFFull) return fail(PT_EINVAL, "sweep counter would exceed 2^32");
  }
  // sweeps-per-cycle candidates: the divisors of the exchange interval up to
  // 16 (any count up to 16 without exchanges), largest first -- the default
  std::vector<uint32_t> Ks;
  for (uint32_t d = 16; d >= 1; --d)
    if (exchange_every ? exchange_every % d == 0 : (d & (d - 1u)) == 0) Ks.push_back(d);
  uint32_t K = Ks[0];
  bool K_tuned = false;
  auto kb = b->K_best.find(exchange_every);
  if (kb != b->K_best.end()) {
    K = kb->second;
    K_tuned = true;
  } else {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    tune_cache_load();
    auto it = g_tuned.find(mix_key(b, exchange_every));
    unsigned k = 0;
    if (it != g_tuned.end() && std::sscanf(it->second.c_str(), "K=%u", &k) == 1 &&
        std::find(Ks.begin(), Ks.end(), k) != Ks.end()) {
      K = k;
      K_tuned = true;
      b->K_best[exchange_every] = K;
    }
  }
  const uint32_t n = (uint32_t)b->ctx.size();
  hipError_t e = hipEventRecord(b->ev_sync, b->user);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->own, b->ev_sync, 0);
  if (e == hipSuccess) e = launch_batch_target(b->d_insts, n, n_sweeps, exchange_every, b->own);
  if (e != hipSuccess) return batch_fail(b, e, "batch start");
  // every instance runs the same schedule: the host replays the sweep count
  // that the device counters reach (a cycle of K runs up to K sweeps and stops
  // at the target and at the next exchange point)
  uint64_t s = b->ctx[0]->sweeps;
  const uint64_t t = s + n_sweeps;
  auto cycle_len = [&](uint32_t k) {
    uint64_t step = std::min<uint64_t>(k, t - s);
    if (exchange_every) step = std::min<uint64_t>(step, exchange_every - s % exchange_every);
    return step;
  };

  // online tuning of the decompositions: untuned groups try one candidate per
  // cycle, timed by events around their sweep launch
  bool tuning = false;
  for (auto &G : b->groups) tuning |= !G.tuned;
  while (tuning && s < t) {
    // groups timing a candidate this cycle: their index and event pair
    std::vector<size_t> timed_groups;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      BatchGroup &G = b->groups[gi];
      if (G.tuned || G.cand_ms.size() >= G.cand.size()) continue;
      const size_t ci = G.cand_ms.size();
      G.W = G.cand[ci].first;
      G.threads = G.cand[ci].second;
      build_items(b, G);
      if ((e = upload_items(b, G, b->own)) != hipSuccess) return batch_fail(b, e, "batch items");
      timed_groups.push_back(gi);
    }
    size_t ti = 0;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      BatchGroup &G = b->groups[gi];
      const bool timed = ti < timed_groups.size() && timed_groups[ti] == gi;
      if (timed && (e = hipEventRecord(b->tune_ev[2 * gi], b->own)) != hipSuccess)
        return batch_fail(b, e, "batch tuning event");
      e = launch_batch_sweep(b->d_insts, b->d_items + G.item_off, (uint32_t)G.items.size(), G.g,
                             G.W, G.threads, K, b->own);
      if (e != hipSuccess) return batch_fail(b, e, "batch sweep launch");
      if (timed) {
        if ((e = hipEventRecord(b->tune_ev[2 * gi + 1], b->own)) != hipSuccess)
          return batch_fail(b, e, "batch tuning event");
        ++ti;
      }
    }
    if ((e = launch_batch_exchange(b->d_insts, b->d_pairs, b->n_pairs, K, b->own)) != hipSuccess ||
        (e = launch_batch_advance(b->d_insts, nullptr, n, K, b->own)) != hipSuccess)
      return batch_fail(b, e, "batch cycle launch");
    s += cycle_len(K);
    if ((e = hipStreamSynchronize(b->own)) != hipSuccess) return batch_fail(b, e, "batch tuning");
    for (size_t gi : timed_groups) {
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, b->tune_ev[2 * gi], b->tune_ev[2 * gi + 1])) != hipSuccess)
        return batch_fail(b, e, "batch tuning timing");
      b->groups[gi].cand_ms.push_back(ms);
    }
    tuning = false;
    for (auto &G : b->groups) {
      if (!G.tuned && G.cand_ms.size() == G.cand.size()) {
        const size_t best = std::min_element(G.cand_ms.begin(), G.cand_ms.end()) - G.cand_ms.begin();
        G.W = G.cand[best].first;
        G.threads = G.cand[best].second;
        G.tuned = true;
        build_items(b, G);
        if ((e = upload_items(b, G, b->own)) != hipSuccess) return batch_fail(b, e, "batch items");
        std::lock_guard<std::mutex> lk(g_tuned_mu);
        tune_cache_put(group_key(b->dev, G.g, G.max_R),
                       "W=" + std::to_string(G.W) + " threads=" + std::to_string(G.threads));
        b->graph_dirty = true;
      }
      tuning |= !G.tuned;
    }
  }

  // online tuning of the sweeps per cycle: one whole graph-replayed cycle per
  // candidate, timed per sweep; only full-length cycles count
  if (!K_tuned && Ks.size() > 1) {
    std::vector<float> per_sweep(Ks.size(), -1.f);
    for (size_t ci = 0; ci < Ks.size() && s < t; ++ci) {
      const uint64_t len = cycle_len(Ks[ci]);
      if (len < Ks[ci]) break; // the rest of the run is shorter than this cycle
      if ((e = batch_graph(b, Ks[ci])) != hipSuccess) return batch_fail(b, e, "batch graph capture");
      if ((e = hipEventRecord(b->tune_ev[0], b->own)) != hipSuccess ||
          (e = hipGraphLaunch(b->exec, b->own)) != hipSuccess ||
          (e = hipEventRecord(b->tune_ev[1], b->own)) != hipSuccess ||
          (e = hipStreamSynchronize(b->own)) != hipSuccess)
        return batch_fail(b, e, "batch cycle timing");
      s += len;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, b->tune_ev[0], b->tune_ev[1])) != hipSuccess)
        return batch_fail(b, e, "batch cycle timing");
      per_sweep[ci] = ms / (float)len;
    }
    if (std::all_of(per_sweep.begin(), per_sweep.end(), [](float v) { return v >= 0.f; })) {
      K = Ks[std::min_element(per_sweep.begin(), per_sweep.end()) - per_sweep.begin()];
      b->K_best[exchange_every] = K;
      std::lock_guard<std::mutex> lk(g_tuned_mu);
      tune_cache_put(mix_key(b, exchange_every), "K=" + std::to_string(K));
    }
  }
  b->K = K;
  if (s < t) {
    if ((e = batch_graph(b, K)) != hipSuccess) return batch_fail(b, e, "batch graph capture");
    while (s < t) {
      if ((e = hipGraphLaunch(b->exec, b->own)) != hipSuccess) return batch_fail(b, e, "batch graph launch");
      s += cycle_len(K);
    }
  }
  if ((e = hipEventRecord(b->ev_sync, b->own)) != hipSuccess ||
      (e = hipStreamWaitEvent(b->user, b->ev_sync, 0)) != hipSuccess)
    return batch_fail(b, e, "batch end");
  for (pt_ctx *c : b->ctx) {
    c->n_records += records_between(c->cfg.record_every, c->sweeps, c->sweeps + n_sweeps);
    if (exchange_every) c->exchanges += records_between(exchange_every, c->sweeps, c->sweeps + n_sweeps);
    c->sweeps += n_sweeps;
  }
  return PT_OK;
}

pt_status pt_batch_observables(pt_batch *b, uint32_t i, pt_obs *obs) {
  if (!b) return fail(PT_EINVAL, "batch is NULL");
  if (b->poisoned) return fail(PT_ESTATE, "batch is poisoned by an earlier device error");
  if (i >= b->ctx.size()) return fail(PT_EINVAL, "instance %u out of range", i);
  hipError_t e = hipStreamSynchronize(b->own);
  uint32_t ctr[kCtrWords];
  if (e == hipSuccess) e = hipMemcpy(ctr, b->d_ctr + (size_t)i * kCtrWords, sizeof ctr, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return batch_fail(b, e, "batch observables");
  pt_ctx *c = b->ctx[i];
  if (ctr[kCtrSweeps] != c->sweeps || ctr[kCtrExchanges] != c->exchanges || ctr[kCtrRecords] != c->n_records) {
    b->poisoned = true;
    return fail(PT_EDEVICE, "instance %u: device schedule (%u sweeps, %u exchanges, %u records) "
                "disagrees with the host (%llu, %llu, %u)", i, ctr[kCtrSweeps], ctr[kCtrExchanges],
                ctr[kCtrRecords], (unsigned long long)c->sweeps, (unsigned long long)c->exchanges,
                c->n_records);
  }
  return pt_observables(c, obs);
}

pt_status pt_batch_group_plan(const pt_batch *b, uint32_t g, uint32_t *L, uint32_t *W,
                              uint32_t *threads, uint32_t *sweeps_per_cycle) {
  if (!b || g >= b->groups.size()) return fail(PT_EINVAL, "group %u out of range", g);
  if (L) *L = b->groups[g].g.L;
  if (W) *W = b->groups[g].W;
  if (threads) *threads = b->groups[g].threads;
  if (sweeps_per_cycle) *sweeps_per_cycle = b->K;
  return PT_OK;
}

void pt_batch_destroy(pt_batch *b) {
  if (!b) return;
  if (b->own) (void)hipStreamSynchronize(b->own);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev_sync) (void)hipEventDestroy(b->ev_sync);
  for (hipEvent_t ev : b->tune_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (b->own) (void)hipStreamDestroy(b->own);
  for (pt_ctx *c : b->ctx) pt_destroy(c);
  delete b;
}

}  // extern "C"
