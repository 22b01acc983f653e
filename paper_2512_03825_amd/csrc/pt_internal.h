// pt_internal.h -- structures shared by the host library (pt_host.cpp) and the
// gfx950 kernels (pt_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptmi {

// Philox purpose tags (counter word 3, bits 8+).
constexpr uint32_t kPurposeFlip = 0u;
constexpr uint32_t kPurposeSwap = 1u << 8;
constexpr uint32_t kPurposeSpin = 2u << 8;
constexpr uint32_t kPurposeBond = 3u << 8;

constexpr uint32_t kClasses = 16;      // flip-threshold classes per slot: 8*b + u
constexpr uint32_t kFieldDigits = 32;  // binary digits of |dM|/2 with a field swap factor
constexpr uint32_t kMaxSweepsPerLaunch = 16;
constexpr uint32_t kMaxParts = 8;            // workgroups per walker of the split persistent plan
// Size of the library's fixed per-GPU scratch array (contexts of pt_create_static).
constexpr size_t kStaticScratchBytes = (size_t)4u << 20;

// Device pointers into the caller's workspace.
struct DevState {
  uint32_t *spins[2];  // [R][N/32] bit-packed, bit set = down (s = -1); walker-indexed
  uint32_t *bonds;     // [3][N/32] bit-packed, bit set = J -1 (EA), bond (i, i+e_d)
  uint32_t *flip_thr;  // [R][16] accept iff r <= T
  uint64_t *flip_cmp;  // [R][16] the same test as an addend: (2^32 - 1) << 32 | ~T, so that
                       // r + entry keeps its high word all ones iff r <= T (else it wraps to 0)
  uint64_t *swap_tab;  // concatenated per-pair tables, accept iff r < T
  uint32_t *swap_off;  // [R] index in swap_tab of pair k's entry d = -D[k]
  uint32_t *swap_D;    // [R] half-width D[k]
  uint64_t *swap_sat;  // [R][2] T for d < -D, T for d > D
  uint32_t swap_n;     // entries in swap_tab
  uint64_t *field_thr; // [R][kFieldDigits] per pair: accept digit j iff r < T (h != 0 only)
  int32_t *field_sign; // [R] sign of (beta_k - beta_k+1) * (-h): the field factor applies when sign * dM < 0
  uint32_t *walker_at; // [R] slot -> walker
  uint32_t *slot_of;   // [R] walker -> slot
  int32_t *E;          // [R] walker E_int
  int32_t *M;          // [R] walker magnetisation
  int32_t *acc3;       // [kMaxSweepsPerLaunch][R][4] per-sweep accumulators (n, sum b, sum cls, -)
  uint32_t *att;       // [R] pair attempts
  uint32_t *acc;       // [R] pair accepts
  int32_t *E_series;   // [max_records][R] slot order
  int32_t *M_series;
  uint32_t *counter;   // [4] workgroup-arrival counter of the tiled sweep; [1] persistent-kernel abort flag
  uint64_t *mailbox;   // [4][R][P][2] persistent kernels (P <= kMaxParts workgroups per walker):
                       // (step + 1) << 32 | E_int share, then M share, posted by the holder of a slot
  uint64_t *halo;      // [2][R][P][split_post_words(g)] split persistent plan: per sweep and part,
                       // (sweep + 1) << 32 | word: boundary planes (bit-packed), then E_int and M shares
  uint8_t *staging;    // +-1 bytes uploaded by the host (only if the config uploads)
};

struct Geometry {
  uint32_t dim;        // 2 or 3
  uint32_t L;
  uint32_t R;
  uint32_t N;          // sites per replica
  uint32_t gpr;        // 8-site groups per row = L/8
  uint32_t rows;       // rows per plane: 1 (2D) or L (3D)
  uint32_t plane;      // bytes per plane = L*rows
  uint32_t nwr;        // packed 32-bit words per walker = ceil(N/32)
  uint32_t phased;     // 2D rows that are not whole 8-site groups, or L not a power of two:
                       // only the phased whole-replica kernel runs it
};

struct Keys {
  uint32_t k0, k1;     // flip / swap / spin stream key
  uint32_t b0;         // bond stream key word 0
};

// Bookkeeping for sweeps, records and exchanges done inside one launch.
struct Schedule {
  uint32_t s0;           // first sweep of the launch
  uint32_t nsw;          // sweeps in the launch
  uint32_t record_every; // 0 = never
  uint32_t rec_base;     // index of the next record
  uint32_t exchange_every; // fused kernel: exchange after sweep s when (s+1) % every == 0
  uint32_t do_exchange;  // tiled kernel: one exchange step after the last sweep
  uint32_t ex_step;      // index e of the next exchange step
};

// ---- batched form: many independent instances advanced together ----------
// Device-resident schedule of one instance (uint32 each).
enum BatchCtr : uint32_t {
  kCtrSweeps = 0,    // sweeps done
  kCtrExchanges = 1, // exchange steps done
  kCtrRecords = 2,   // records written
  kCtrTarget = 3,    // run until this many sweeps are done
  kCtrActive = 4,    // 0: the instance is idle
  kCtrEvery = 5,     // exchange interval (0 = never)
  kCtrCur = 6,       // tiled instances: spin buffer holding the lattices
  kCtrTiles = 7,     // tiled instances: tiles per walker (0: whole replicas in LDS)
  kCtrWords = 8
};

struct BatchInst {
  DevState st;
  Geometry geo;
  Keys key;
  uint32_t record_every;
  uint32_t lg_L, lg_spr, lg_rows, lg_items; // as in the fused kernel, for span_groups(geo)
  int32_t z2;
  uint32_t *ctr; // [kCtrWords]
};

struct BatchItem {
  uint32_t inst; // instance index
  uint32_t w0;   // first walker of the workgroup (up to W walkers)
};

// Work item of the batched tiled sweep: one tile of one walker of an instance.
struct BatchTileItem {
  uint32_t inst, w, tile, pad;
};

// One cycle of at most K sweeps: sweep launches (one per lattice-size group),
// then the exchange launch, then the counter advance.
hipError_t launch_batch_sweep(const BatchInst *insts, const BatchItem *items, uint32_t n_items,
                              const Geometry &g, uint32_t W, uint32_t threads, uint32_t K,
                              hipStream_t stream);
hipError_t launch_batch_exchange(const BatchInst *insts, const uint2 *pairs, uint32_t n_pairs,
                                 uint32_t K, hipStream_t stream);
// Advance the schedule counters of instances list[0 .. n) (list = NULL: 0 .. n).
hipError_t launch_batch_advance(const BatchInst *insts, const uint32_t *list, uint32_t n_insts,
                                uint32_t K, hipStream_t stream);
// Batched 2D tiled sweep: items of instances of one lattice size L, tiles of H
// rows, up to K sweeps per instance (to its next exchange point); each
// instance's last workgroup folds E and M, records and exchanges.
hipError_t launch_batch_tiled(const BatchInst *insts, const BatchTileItem *items, uint32_t n_items,
                              const Geometry &g, uint32_t H, uint32_t threads, uint32_t K,
                              hipStream_t stream);
size_t batch_lds_bytes(const Geometry &g, uint32_t W);
// Start a run: every instance's target = done + add, active if add > 0, interval = every.
hipError_t launch_batch_target(const BatchInst *insts, uint32_t n, uint32_t add, uint32_t every,
                               hipStream_t stream);

hipError_t launch_init_spins(const DevState &st, const Geometry &g, const Keys &k, bool upload,
                             hipStream_t stream);
hipError_t launch_init_bonds(const DevState &st, const Geometry &g, const Keys &k, bool upload,
                             hipStream_t stream);
hipError_t launch_reset(const DevState &st, const Geometry &g, hipStream_t stream);
hipError_t launch_recount(const DevState &st, const Geometry &g, uint32_t cur,
                          hipStream_t stream);
hipError_t launch_exchange(const DevState &st, const Geometry &g, const Keys &k, uint32_t e,
                           hipStream_t stream);
hipError_t launch_tiled(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                        uint32_t tile_planes, uint32_t halo, uint32_t threads,
                        const Schedule &sch, hipStream_t stream);
hipError_t launch_fused(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                        uint32_t threads, const Schedule &sch, hipStream_t stream);
// One lane per walker, whole lattice in registers (2D, L = 8 or 16, R <= 1024).
hipError_t launch_lanes(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                        const Schedule &sch, hipStream_t stream);
size_t lanes_lds_bytes(const Geometry &g);
// Each walker in the registers of L^2/8 lanes of one wavefront, one nibble
// dword per lane (2D, L = 8 or 16, R L^2/8 <= 1024 threads), one workgroup.
hipError_t launch_wave(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                       const Schedule &sch, hipStream_t stream);
size_t wave_lds_bytes(const Geometry &g);
uint32_t wave_threads(const Geometry &g);
// One co-resident workgroup per walker (parts = 1), or in 3D two per walker,
// each holding half of the z-planes (parts = 2), for the whole launch; exchange
// decisions are taken pairwise through per-slot mailboxes (cooperative launch).
hipError_t launch_persist(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                          uint32_t threads, uint32_t parts, const Schedule &sch,
                          uint32_t spin_limit, hipStream_t stream);
// Words one part of a split walker posts per sweep: its two lowest and two
// highest planes (3D z-planes, 2D rows) bit-packed, then its E_int and M shares.
inline uint32_t split_post_words(const Geometry &g) { return 4u * (g.plane / 32u) + 2u; }
// Workgroups per walker the split plan allows: 3D 16 <= L <= 32 two (L/2
// z-planes each); 2D 64 <= L <= 1024 up to kMaxParts (rows); 0 otherwise.
inline uint32_t split_max_parts(const Geometry &g) {
  if (g.dim == 3) return (g.L >= 16u && g.L <= 32u) ? 2u : 0u;
  return (g.L >= 64u && g.L <= 1024u) ? kMaxParts : 0u;
}
// uint64 words of the post area: two generations of every part's post.
inline size_t split_halo_words(const Geometry &g) {
  return (size_t)2u * g.R * split_max_parts(g) * split_post_words(g);
}

// Groups of 8 sites one lane updates per item (V): 2D min(4, L/8), 3D min(2, L/8).
uint32_t span_groups(const Geometry &g);
// The same for the batched kernels: 2D min(8, L/8), 3D min(2, L/8).
uint32_t batch_span(const Geometry &g);

// LDS bytes needed by the kernels (host-side planning).
size_t tiled_lds_bytes(const Geometry &g, uint32_t tile_planes, uint32_t halo);
// LDS of the phased whole-replica kernel (2D lattices with g.phased set).
size_t phased_lds_bytes(const Geometry &g);
size_t fused_lds_bytes(const Geometry &g);
size_t persist_lds_bytes(const Geometry &g, uint32_t parts);
// Workgroups of the persistent kernel that can be co-resident (0 if unknown).
uint32_t persist_max_workgroups(const Geometry &g, uint32_t threads, uint32_t parts);
size_t max_lds_bytes();

// The current device's copy of the library's fixed scratch array
// (kStaticScratchBytes, 256-byte aligned): its device address, looked up once
// per device with that device current.
hipError_t static_scratch(uint8_t **out);
// Zero `bytes` (a multiple of 8) of device memory at p with a fill kernel (no
// memset node, so the call may be captured in a graph).
hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream);

}  // namespace ptmi
