// pt_host.h -- host-side structures shared by the library's C ABI files
// (pt_host.cpp: plain and batched forms; pt_serve.cpp: served form).  Not part
// of the public ABI.
#pragma once

#include "pt.h"
#include "pt_internal.h"

#include <memory>
#include <utility>
#include <vector>

namespace ptmi {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Records the message for pt_last_error() and returns st.
pt_status fail(pt_status st, const char *fmt, ...);
// Multiples of `every` in (s0, s1] (0 when every = 0).
uint32_t records_between(uint32_t every, uint64_t s0, uint64_t s1);
uint32_t lg2(uint32_t v);

struct Tables {
  std::vector<uint32_t> flip; // [R][16]
  std::vector<uint64_t> flipc; // [R][16] the kernels' form of flip: (2^32 - 1) << 32 | ~T
  std::vector<uint64_t> swap; // concatenated pair tables
  std::vector<uint32_t> off;  // [R]
  std::vector<uint32_t> D;    // [R]
  std::vector<uint64_t> sat;  // [R][2]
  std::vector<uint64_t> field; // [R][kFieldDigits]
  std::vector<int32_t> fsign;  // [R]
};

// Byte offsets in a context's workspace.  The scratch of the sweep kernels
// (per-sweep tallies, exchange mailboxes, boundary posts) comes last, from
// offset `scratch` to `total`, so that a context whose scratch lives in the
// library's fixed array (pt_create_static) needs only the first `scratch` bytes.
struct Layout {
  size_t spins[2], bonds, staging, flip, flipc, swap_tab, swap_off, swap_D, swap_sat, wat, sof, E, M,
      att, acc, Es, Ms, counter, field, fsign, scratch, acc3, mailbox, halo, total;
};

struct Derived {
  Geometry geo;
  double jscale; // energy unit of E_int: J (2D), 1 (EA)
  uint32_t z;    // coordination number
};

}  // namespace ptmi

using ptmi::Derived;
using ptmi::DevState;
using ptmi::Keys;
using ptmi::Layout;
using ptmi::Tables;

struct pt_ctx {
  pt_config cfg;
  std::vector<double> beta;
  Derived d;
  Keys keys;
  DevState st;
  Layout lay;
  std::shared_ptr<const Tables> tab; // shared with contexts of the same ladder
  hipStream_t stream;
  pt_plan plan;
  uint64_t sweeps = 0, exchanges = 0;
  uint32_t n_records = 0;
  uint32_t cur = 0;
  // polls of a partner's post (each followed by a short sleep) before a
  // persistent launch gives up: orders of magnitude above any legitimate wait
  uint32_t wait_limit = 1u << 24;
  bool poisoned = false;
  // pt_create_static: the device's fixed scratch array holds acc3, mailbox and
  // halo (cleared before every sweep call); NULL: they are in the workspace
  uint8_t *static_scratch = nullptr;
};

namespace ptmi {

// pt_create with a choice: sync = false leaves the initialisation kernels
// queued on the stream (errors then surface at the next synchronisation);
// static_scratch != NULL places the scratch regions there instead of in the
// workspace (which then needs only Layout::scratch bytes).
pt_status ctx_create(const pt_config *cfg, hipStream_t stream, void *d_workspace, size_t ws_bytes,
                     bool sync, uint8_t *static_scratch, pt_ctx **out);
// Queue n sweeps of the context's plan; exchange after sweep s when every > 0
// and (s+1) % every == 0.
pt_status ctx_advance(pt_ctx *c, uint32_t n, uint32_t every);
// Device descriptor of a context for the batched kernels; ctr = its counters.
BatchInst batch_inst(const pt_ctx *c, uint32_t *ctr);
// Whole replicas of this geometry fit one workgroup's LDS (batched kernels).
bool batch_fits(const Geometry &g);
// Walkers per workgroup and threads for a batched group of this geometry: the
// decomposition tuned earlier in this process if there is one, else a default.
std::pair<uint32_t, uint32_t> batch_decomposition(const Geometry &g, uint32_t max_R);

}  // namespace ptmi
