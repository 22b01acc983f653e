// pt_kernels.hip -- gfx950 kernels of the parallel-tempering Metropolis library.
//
// Lattices live bit-packed in HBM (bit set = down spin) and are unpacked into
// LDS at four bits per site: a row of L sites is L/8 dwords, one dword per
// group of 8 sites (EA bonds: three more such arrays, bond (i, i+e_d) at site
// i).  A value of 0 is an up spin (s = +1) and 1 a down spin, so the number of
// unsatisfied bonds of a site is a nibble-wise sum of XORs with its neighbours
// (at most 6, no carries between nibbles).  In a group the four sites of the
// colour being updated sit at nibbles off, off+2, off+4, off+6 (off = colour
// parity of the row) and consume the four words of one Philox4x32-10 block
// whose counter is the group's index: the draw of site i is word (i/2) mod 4
// of block (i/2)/4, as the method's draw mapping fixes.
//
// Work of one group: the neighbour dwords from LDS, a SWAR count of
// unsatisfied bonds, one Philox block (18 vector 64-bit multiplies + 20
// three-way XORs), four LDS threshold lookups and compares, one store, and the
// exact integer energy / magnetisation change of the accepted flips (v_dot8
// tallies over nibbles).
//
// Kernels:
//   k_tiled_n      2D, grid (tiles, walkers).  A workgroup stages one tile of
//   k_tiled<3>     rows (z-planes in 3D) plus halo rows of its walker in LDS
//                  and runs up to 8 sweeps on it.  With halo depth 2k for k
//                  sweeps the interior stays exact (every half sweep
//                  recomputes one row less on each side with the same draws);
//                  tiles read one spin buffer and write the other.  A
//                  whole-replica tile (halo 0) updates in place.  The last
//                  workgroup to finish folds the per-sweep energy changes into
//                  E and M, writes the records, and runs the exchange step.
//   k_fused        one workgroup holds every walker of a small system in LDS
//                  and runs sweeps, records and exchange steps without leaving
//                  the kernel.
//   k_persist      one co-resident workgroup per walker for a whole run;
//                  exchanges decided pairwise through mailboxes.
//   k_persist_split  P co-resident workgroups per walker (L/P z-planes in 3D,
//                  rows in 2D, two halo planes per side), trading boundary
//                  planes and energy shares once per sweep as tagged words.
//   k_wave         small 2D lattices: each walker in the registers of the
//                  lanes of one wavefront (a nibble dword per lane), neighbours
//                  by cross-lane reads, no barrier within a sweep.
//   k_lanes        the paper's decomposition: one walker per lane, its lattice
//                  in registers, sites visited one after another.
//   k_batch_*      batched and served forms: many instances per launch.
//   k_exchange     one exchange step (slot permutation, no lattice copies).
//   k_init_*, k_reset, k_recount   initialisation.
#include "pt_internal.h"

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

// Scratch of the contexts made by pt_create_static (per-sweep tallies, exchange
// mailboxes, boundary posts): one copy per GPU, resident until the process
// ends.  In host code this name is not a device address; the address is taken
// once per device with hipGetSymbolAddress (static_scratch below).
static __device__ __align__(256) uint8_t scratch[ptmi::kStaticScratchBytes];

namespace ptmi {
namespace {

constexpr int kMaxThreads = 1024;
// Groups (dwords) one lane updates per item: the 2D tiled kernel (chosen by
// measurement among 2, 4, 8) and the persistent kernel (among 2, 4).
constexpr uint32_t kNibbleSpan = 8;
constexpr uint32_t kPersistSpan = 4;
// Words a split-plan part reads per sweep, per lane of the reading wave: the
// boundary planes (4 x 32 packed words for 3D L <= 32 and 2D L <= 1024) and
// 2 (P - 1) shares, at most 142 words over 64 lanes.
constexpr uint32_t kSplitWordsPerLane = 3;

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// (a ^ b) + c in one VALU instruction.
__device__ __forceinline__ uint32_t xad(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t d;
  asm("v_xad_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

struct Words {
  uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 products,
// Weyl key schedule between rounds.
__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// Sweeps of this cycle for an instance: at most K, never past the target, and
// never past the next exchange point (a cycle always ends on one).
__device__ __forceinline__ uint32_t cycle_sweeps(const uint32_t *ctr, uint32_t K) {
  if (!ctr[kCtrActive]) return 0u;
  const uint32_t s = ctr[kCtrSweeps], every = ctr[kCtrEvery];
  uint32_t n = min(K, ctr[kCtrTarget] - s);
  if (every) n = min(n, every - s % every);
  return n;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Sum of v over each aligned group of 16 lanes (DPP row rotations, every lane
// ends with its row's sum).
__device__ __forceinline__ int row_sum16(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x121, 0xF, 0xF, false); // row_ror:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x122, 0xF, 0xF, false); // row_ror:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x124, 0xF, 0xF, false); // row_ror:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false); // row_ror:8
  return v;
}

// The value of lane l ^ 16 (ds_swizzle, bit-mask mode: and 0x1F, or 0, xor 0x10).
__device__ __forceinline__ int swap16(int v) { return __builtin_amdgcn_ds_swizzle(v, 0x401F); }

// Sum of v over the whole wavefront, uniform (read into a scalar register):
// DPP row sums, then the four rows' sums lane by lane -- no LDS-unit permutes
// on the way.  Every lane must be active.
__device__ __forceinline__ int wave_total(int v) {
  v = row_sum16(v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

// The swap-test tables as one kernel reads them: in device memory, or copies
// in LDS (the fused kernel stages them when they are small).
struct SwapView {
  const uint64_t *tab; // concatenated per-pair rows
  const uint32_t *off; // [R] row start of pair k (entry d = -D[k])
  const uint32_t *D;   // [R] half-width of pair k's row
  const uint64_t *sat; // [R][2] values for d < -D and d > D
  uint32_t n;          // entries in tab
};

// The part of pair k's swap table that does not depend on the energies: its
// half-width, row start and two saturation values.  Loaded ahead (before a
// wait, beside the walker map), so that the test itself is one table read.
struct PairRow {
  int32_t D;
  uint32_t off;
  uint64_t lo, hi;
};

__device__ __forceinline__ PairRow pair_row(const SwapView &v, uint32_t k) {
  return PairRow{(int32_t)v.D[k], v.off[k], v.sat[2u * k], v.sat[2u * k + 1u]};
}
__device__ __forceinline__ PairRow pair_row(const DevState &st, uint32_t k) {
  return PairRow{(int32_t)st.swap_D[k], st.swap_off[k], st.swap_sat[2u * k], st.swap_sat[2u * k + 1u]};
}

// Threshold of the pair for E_a - E_b (E_int at slots k, k+1): accept iff r < T.
__device__ __forceinline__ uint64_t pair_T(const PairRow &p, const uint64_t *tab, uint32_t n,
                                           int32_t dEint) {
  const int32_t d = dEint / 4; // E_int differences are multiples of 4
  if (d < -p.D) return p.lo;
  if (d > p.D) return p.hi;
  const uint32_t idx = p.off + (uint32_t)(d + p.D);
  return idx < n ? tab[idx] : 0u; // a valid table always passes
}

__device__ __forceinline__ uint64_t swap_T(const SwapView &v, uint32_t k, int32_t dEint) {
  return pair_T(pair_row(v, k), v.tab, v.n, dEint);
}

// Field factor of a swap (2D, h != 0): with y = (beta_k - beta_k+1)(-h) dM < 0,
// one Metropolis test per set binary digit j of |dM|/2, each with its own draw
// (word j mod 4 of block (k, e, 1 + j/4, swap purpose)).
__device__ __forceinline__ bool field_factor(const DevState &st, int32_t sg, uint32_t k,
                                             uint32_t e, int32_t dM, uint32_t k0, uint32_t k1) {
  if (sg == 0 || dM == 0 || (sg > 0) == (dM > 0)) return true; // y >= 0
  const uint32_t n = (uint32_t)(dM < 0 ? -dM : dM) >> 1;
  for (uint32_t j = 0; j < kFieldDigits && (n >> j); ++j) {
    if (!((n >> j) & 1u)) continue;
    const Words w = philox(k, e, 1u + (j >> 2), kPurposeSwap, k0, k1);
    const uint32_t r = (j & 3u) == 0 ? w.x : (j & 3u) == 1 ? w.y : (j & 3u) == 2 ? w.z : w.w;
    if ((uint64_t)r >= st.field_thr[(size_t)k * kFieldDigits + j]) return false;
  }
  return true;
}

// Exchange decision for the pair of slots (k, k+1) at step e; on acceptance the
// two walkers trade slots.  Counts the attempt and the acceptance.
__device__ __forceinline__ void exchange_pair(const DevState &st, uint32_t k, uint32_t k0,
                                              uint32_t k1, uint32_t e, const int32_t *E,
                                              const int32_t *M, uint32_t *walker_at,
                                              uint32_t *slot_of) {
  // the pair's table data does not depend on the energies: loaded together
  // with the walker map, so the test costs three dependent memory accesses
  const uint32_t a = walker_at[k], b = walker_at[k + 1u];
  const PairRow row = pair_row(st, k);
  const int32_t sg = st.field_sign[k];
  const uint32_t r = philox(k, e, 0u, kPurposeSwap, k0, k1).x;
  const uint64_t T = pair_T(row, st.swap_tab, st.swap_n, E[a] - E[b]);
  atomicAdd(&st.att[k], 1u); // one lane per pair: the atomic only spares a round trip
  if ((uint64_t)r < T && field_factor(st, sg, k, e, M[a] - M[b], k0, k1)) {
    walker_at[k] = b;
    walker_at[k + 1u] = a;
    slot_of[a] = k + 1u;
    slot_of[b] = k;
    atomicAdd(&st.acc[k], 1u);
  }
}

// One exchange step with parity e & 1 on the given walker/slot maps.
__device__ void exchange_step(const DevState &st, uint32_t R, uint32_t k0, uint32_t k1,
                              uint32_t e, const int32_t *E, const int32_t *M,
                              uint32_t *walker_at, uint32_t *slot_of, uint32_t tid, uint32_t nt) {
  for (uint32_t k = (e & 1u) + 2u * tid; k + 1u < R; k += 2u * nt)
    exchange_pair(st, k, k0, k1, e, E, M, walker_at, slot_of);
}

struct TiledArgs {
  DevState st;
  Geometry geo;
  Keys key;
  Schedule sch;
  const uint32_t *src; // bit-packed spins read by this launch
  uint32_t *dst;       // bit-packed spins written by this launch
  uint32_t H;      // interior planes per tile (last tile may be shorter)
  uint32_t halo;   // halo planes per side (0 = whole replica, in place)
  uint32_t lg_L;   // log2(L)
  uint32_t lg_spr; // log2(spans per row) = log2(L / (8 V))
  uint32_t lg_rows;
  int32_t z2;      // 2 * coordination number (8 in 2D, 12 in 3D)
};

// The last workgroup of a tiled launch to arrive folds the per-sweep energy
// and magnetisation changes into E and M, writes the records, and runs the
// exchange step; it then re-arms the arrival counter.
// total = workgroups of the launch working on this walker set.
__device__ __forceinline__ void tiled_epilogue(const TiledArgs &a, uint32_t tid, uint32_t nt,
                                               uint32_t *s_last, uint32_t total) {
  __syncthreads();
  if (tid == 0u) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); // publish this workgroup's tallies
    const uint32_t prev =
        __hip_atomic_fetch_add(a.st.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    *s_last = (prev + 1u == total) ? 1u : 0u;
  }
  __syncthreads();
  if (!*s_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

  // Each thread folds whole walkers: every load of a walker (its per-sweep
  // tallies, E, M, slot) is issued before any is used, so the fold costs one
  // memory round trip whatever the number of sweeps.  The slots do not change
  // before the exchange step, so walker v's record goes to column slot_of[v].
  const uint32_t R = a.geo.R, nsw = a.sch.nsw;
  for (uint32_t v = tid; v < R; v += nt) {
    int32_t dE[kMaxSweepsPerLaunch], dM[kMaxSweepsPerLaunch];
#pragma unroll
    for (uint32_t j = 0; j < kMaxSweepsPerLaunch; ++j) {
      if (j >= nsw) break;
      const int32_t *acc = a.st.acc3 + ((size_t)j * R + v) * 4u;
      dE[j] = __hip_atomic_load(acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      dM[j] = __hip_atomic_load(acc + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int32_t Ev = a.st.E[v], Mv = a.st.M[v];
    const uint32_t k = a.st.slot_of[v];
    uint32_t rec = a.sch.rec_base;
#pragma unroll
    for (uint32_t j = 0; j < kMaxSweepsPerLaunch; ++j) {
      if (j >= nsw) break;
      int32_t *acc = a.st.acc3 + ((size_t)j * R + v) * 4u;
      __hip_atomic_store(acc, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(acc + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      Ev += dE[j];
      Mv += dM[j];
      if (a.sch.record_every && (a.sch.s0 + j + 1u) % a.sch.record_every == 0u) {
        a.st.E_series[(size_t)rec * R + k] = Ev;
        a.st.M_series[(size_t)rec * R + k] = Mv;
        ++rec;
      }
    }
    a.st.E[v] = Ev;
    a.st.M[v] = Mv;
  }
  if (a.sch.do_exchange) {
    __syncthreads();
    exchange_step(a.st, R, a.key.k0, a.key.k1, a.sch.ex_step, a.st.E, a.st.M, a.st.walker_at,
                  a.st.slot_of, tid, nt);
  }
  __syncthreads();
  if (tid == 0u) __hip_atomic_store(a.st.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}



// Whole replicas, one workgroup per walker: the walker is this workgroup's
// alone, so thread 0 folds its per-sweep changes (s_sw) into E and M and writes
// its records (its slot does not change before the exchange step, which runs
// as a launch of its own after the sweeps).
__device__ __forceinline__ void fold_own_walker(const TiledArgs &a, uint32_t w,
                                                const int (*s_sw)[2]) {
  const uint32_t R = a.geo.R, slot = a.st.slot_of[w];
  int32_t E = a.st.E[w], M = a.st.M[w];
  uint32_t rec = a.sch.rec_base;
  for (uint32_t j = 0; j < a.sch.nsw; ++j) {
    E += s_sw[j][0];
    M += s_sw[j][1];
    if (a.sch.record_every && (a.sch.s0 + j + 1u) % a.sch.record_every == 0u) {
      a.st.E_series[(size_t)rec * R + slot] = E;
      a.st.M_series[(size_t)rec * R + slot] = M;
      ++rec;
    }
  }
  a.st.E[w] = E;
  a.st.M[w] = M;
}

// ---- the four-bit LDS layout -------------------------------------------------
// Site 8g + j of a row sits at bits 4j .. 4j+3 of the row's dword g.  A dword
// is exactly one Philox group; a site's class 8b + u fits its nibble, and the
// tallies are v_dot8 products over nibbles.

// 8 bits -> 8 nibbles (bit j -> bit 4j), and back.
__device__ __forceinline__ uint32_t spread8(uint32_t x) {
  x = (x | (x << 12)) & 0x000F000Fu;
  x = (x | (x << 6)) & 0x03030303u;
  return (x | (x << 3)) & 0x11111111u;
}
__device__ __forceinline__ uint32_t gather8(uint32_t x) {
  x &= 0x11111111u;
  x = (x | (x >> 3)) & 0x03030303u;
  x = (x | (x >> 6)) & 0x000F000Fu;
  return (x | (x >> 12)) & 0x000000FFu;
}

// LDS dwords [4q, 4q + 4) <- nibbles of packed words src[(f + q) & m], q < cnt.
__device__ __forceinline__ void unpack_tile_n(uint32_t *lds, const uint32_t *src, uint32_t f,
                                              uint32_t cnt, uint32_t m, uint32_t tid, uint32_t nt) {
  constexpr uint32_t kBatch = 4;
  for (uint32_t q0 = tid; q0 < cnt; q0 += kBatch * nt) {
    uint32_t w[kBatch];
#pragma unroll
    for (uint32_t j = 0; j < kBatch; ++j) {
      const uint32_t q = q0 + j * nt;
      w[j] = (q < cnt) ? src[(f + q) & m] : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kBatch; ++j) {
      const uint32_t q = q0 + j * nt;
      if (q < cnt)
        reinterpret_cast<uint4 *>(lds)[q] =
            make_uint4(spread8(w[j] & 0xFFu), spread8(__builtin_amdgcn_ubfe(w[j], 8u, 8u)),
                       spread8(__builtin_amdgcn_ubfe(w[j], 16u, 8u)), spread8(w[j] >> 24));
    }
  }
}

// dst[q] <- packed nibbles of LDS dwords [4q, 4q + 4), q < cnt.
__device__ __forceinline__ void pack_tile_n(uint32_t *dst, const uint32_t *lds, uint32_t cnt,
                                            uint32_t tid, uint32_t nt) {
  for (uint32_t q = tid; q < cnt; q += nt) {
    const uint4 x = reinterpret_cast<const uint4 *>(lds)[q];
    dst[q] = gather8(x.x) | (gather8(x.y) << 8) | (gather8(x.z) << 16) | (gather8(x.w) << 24);
  }
}

template <int V>
__device__ __forceinline__ void lds_load_n(uint32_t (&d)[V], const uint32_t *p) {
  if constexpr (V == 8) {
    const uint4 a = reinterpret_cast<const uint4 *>(p)[0], b = reinterpret_cast<const uint4 *>(p)[1];
    d[0] = a.x;
    d[1] = a.y;
    d[2] = a.z;
    d[3] = a.w;
    d[4] = b.x;
    d[5] = b.y;
    d[6] = b.z;
    d[7] = b.w;
  } else if constexpr (V == 4) {
    const uint4 a = *reinterpret_cast<const uint4 *>(p);
    d[0] = a.x;
    d[1] = a.y;
    d[2] = a.z;
    d[3] = a.w;
  } else if constexpr (V == 2) {
    const uint2 a = *reinterpret_cast<const uint2 *>(p);
    d[0] = a.x;
    d[1] = a.y;
  } else {
    d[0] = p[0];
  }
}
template <int V>
__device__ __forceinline__ void lds_store_n(uint32_t *p, const uint32_t (&d)[V]) {
  if constexpr (V == 8) {
    reinterpret_cast<uint4 *>(p)[0] = make_uint4(d[0], d[1], d[2], d[3]);
    reinterpret_cast<uint4 *>(p)[1] = make_uint4(d[4], d[5], d[6], d[7]);
  } else if constexpr (V == 4)
    *reinterpret_cast<uint4 *>(p) = make_uint4(d[0], d[1], d[2], d[3]);
  else if constexpr (V == 2)
    *reinterpret_cast<uint2 *>(p) = make_uint2(d[0], d[1]);
  else
    p[0] = d[0];
}

// Tallies of the nibble layout: n flips, sb = down spins flipped, sc = sum of
// the flipped sites' classes 8b + u.
struct TallyN {
  uint32_t n, sb, sc;
};

// High word of r + c (64-bit): one v_mad_u64_u32 (r * 1 + c).  With a table
// entry c = (2^32 - 1) << 32 | ~T it is all ones iff r <= T and 0 otherwise,
// so the flip test leaves its outcome as a mask in a vector register.
__device__ __forceinline__ uint32_t carry_mask(uint32_t r, uint64_t c) {
  // a multiplier of 1 the compiler cannot see through (else it would fold the
  // product away and add in two instructions); set once, kept in a scalar register
  uint32_t one;
  asm("s_mov_b32 %0, 1" : "=s"(one));
  return (uint32_t)(((uint64_t)r * one + c) >> 32);
}

// Metropolis decision for the four colour sites of one dword (nibble layout):
// w = spins, u = unsatisfied-bond counts per nibble, r = the group's draws,
// tb = the slot's 16 table entries.  Returns the new spins and adds the
// accepted flips to the tallies.
//   WIDE: 8-byte entries in the flip_cmp form, tested by the carry of r + entry
//         (4 multiply-adds, 2 byte permutes and one three-input op for the four
//         sites: 7 instructions, against 10 for compares and selects);
//   else: 4-byte thresholds T, tested by r <= T (half the LDS bytes; measured
//         faster in the 2D split kernel, whose 16 waves per compute unit hide
//         less LDS latency than the tiled, phased and 3D kernels' 24).
// vm: nibbles that are sites (low bit of each nibble set); padding nibbles
// never flip.
template <bool WIDE>
__device__ __forceinline__ uint32_t decide_n(uint32_t w, uint32_t u, uint32_t off, const Words &r,
                                             const uint8_t *tb, TallyN &t,
                                             uint32_t vm = 0xFFFFFFFFu) {
  const uint32_t M = off ? 0xF0F0F0F0u : 0x0F0F0F0Fu;   // colour nibbles
  const uint32_t cls = ((w << 3) | u) & M;              // 8b + u in each colour nibble
  uint32_t f;
  if constexpr (WIDE) {
    const uint32_t rot = off ? 1u : 29u;                // class * 8 to bits 8m .. 8m+6
    const uint32_t c8 = __builtin_amdgcn_alignbit(cls, cls, rot);
    const uint64_t t0 = *reinterpret_cast<const uint64_t *>(tb + (c8 & 0xFFu));
    const uint64_t t1 = *reinterpret_cast<const uint64_t *>(tb + __builtin_amdgcn_ubfe(c8, 8u, 8u));
    const uint64_t t2 = *reinterpret_cast<const uint64_t *>(tb + __builtin_amdgcn_ubfe(c8, 16u, 8u));
    const uint64_t t3 = *reinterpret_cast<const uint64_t *>(tb + (c8 >> 24));
    // accept masks (all ones or 0) of the four sites, their low bytes gathered
    // into bytes 0..3, then the colour nibbles' low bits kept
    const uint32_t a01 = __builtin_amdgcn_perm(carry_mask(r.y, t1), carry_mask(r.x, t0), 0x0C0C0400u);
    const uint32_t a23 = __builtin_amdgcn_perm(carry_mask(r.w, t3), carry_mask(r.z, t2), 0x04000C0Cu);
    f = __builtin_amdgcn_bitop3_b32(a01, a23, (0x01010101u << (4u * off)) & vm, 0xA8); // (a | b) & c
  } else {
    const uint32_t rot = off ? 2u : 30u;                // class * 4 to bits 8m .. 8m+5
    const uint32_t b0 = 1u << (4u * off);
    const uint32_t c4 = __builtin_amdgcn_alignbit(cls, cls, rot);
    const uint32_t t0 = *reinterpret_cast<const uint32_t *>(tb + (c4 & 63u));
    const uint32_t t1 = *reinterpret_cast<const uint32_t *>(tb + __builtin_amdgcn_ubfe(c4, 8u, 6u));
    const uint32_t t2 = *reinterpret_cast<const uint32_t *>(tb + __builtin_amdgcn_ubfe(c4, 16u, 6u));
    const uint32_t t3 = *reinterpret_cast<const uint32_t *>(tb + (c4 >> 24));
    f = ((r.x <= t0 ? b0 : 0u) | (r.y <= t1 ? (b0 << 8) : 0u) | (r.z <= t2 ? (b0 << 16) : 0u) |
         (r.w <= t3 ? (b0 << 24) : 0u)) & vm;
  }
  t.n += __builtin_popcount(f);
  t.sb = __builtin_amdgcn_udot8(w, f, t.sb, false);
  t.sc = __builtin_amdgcn_udot8(cls, f, t.sc, false);
  return w ^ f;
}

// 2D Ising, nibble layout: update the colour sites of the V groups (dwords)
// g0 .. g0+V-1 of one row.
template <int V, bool WIDE = true>
__device__ __forceinline__ void span2d_n(uint32_t *row, const uint32_t *up, const uint32_t *dn,
                                         uint32_t g0, uint32_t gmask, uint32_t off,
                                         const Words (&r)[V], const void *thr, TallyN &t) {
  uint32_t w[V], a[V], b[V], nw[V];
  lds_load_n<V>(w, row + g0);
  lds_load_n<V>(a, up + g0);
  lds_load_n<V>(b, dn + g0);
  // the neighbouring dword on the side the colour sites need: left for off = 0
  // (nibble 0's left neighbour), right for off = 1 (nibble 7's right neighbour)
  const uint32_t e = row[off ? ((g0 + V) & gmask) : ((g0 + gmask) & gmask)];
  const uint8_t *tb = reinterpret_cast<const uint8_t *>(thr);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint32_t l = __builtin_amdgcn_alignbit(w[v], v ? w[v - 1] : e, 28u);
    const uint32_t rr = __builtin_amdgcn_alignbit(v < V - 1 ? w[v + 1] : e, w[v], 4u);
    uint32_t u = rr ^ w[v];
    u = xad(l, w[v], u);
    u = xad(b[v], w[v], u);
    u = xad(a[v], w[v], u);
    nw[v] = decide_n<WIDE>(w[v], u, off, r[v], tb, t);
  }
  lds_store_n<V>(row + g0, nw);
}

// 3D +-J EA, nibble layout: spins and the three bond planes (bond (i, i+e_d)
// at site i, bit set = J -1) are dword arrays with plane p, row y at dword
// (p << lgPl) + (y << lgG).  Updates the colour sites of V dwords g0.. of row
// y of plane pl; a bond is unsatisfied iff s_i ^ s_j ^ J_ij = 1.
template <int V, bool WIDE = true>
__device__ __forceinline__ void span3d_n(uint32_t *sp, const uint32_t *bx, const uint32_t *by,
                                         const uint32_t *bz, uint32_t lgG, uint32_t lgPl,
                                         uint32_t pl, uint32_t pu, uint32_t pd, uint32_t y,
                                         uint32_t yu, uint32_t yd, uint32_t g0, uint32_t gmask,
                                         uint32_t off, const Words (&r)[V], const void *thr,
                                         TallyN &t) {
  const uint32_t rowb = (pl << lgPl) + (y << lgG);
  uint32_t w[V], jx[V], u[V], nw[V];
  lds_load_n<V>(w, sp + rowb + g0);
  lds_load_n<V>(jx, bx + rowb + g0);
  const uint32_t eg = rowb + (off ? ((g0 + V) & gmask) : ((g0 + gmask) & gmask));
  const uint32_t es = sp[eg];
  const uint32_t ej = off ? 0u : bx[eg];   // +x bond of the left neighbour (off = 0 only)
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint32_t l = __builtin_amdgcn_alignbit(w[v], v ? w[v - 1] : es, 28u);
    const uint32_t lj = __builtin_amdgcn_alignbit(jx[v], v ? jx[v - 1] : ej, 28u);
    const uint32_t rr = __builtin_amdgcn_alignbit(v < V - 1 ? w[v + 1] : es, w[v], 4u);
    u[v] = xor3(l, w[v], lj) + xor3(rr, w[v], jx[v]);
  }
  {
    uint32_t s0[V], s1[V], j0[V], j1[V];
    lds_load_n<V>(s0, sp + (pl << lgPl) + (yu << lgG) + g0);   // row y-1
    lds_load_n<V>(s1, sp + (pl << lgPl) + (yd << lgG) + g0);   // row y+1
    lds_load_n<V>(j0, by + (pl << lgPl) + (yu << lgG) + g0);   // its +y bond to us
    lds_load_n<V>(j1, by + rowb + g0);
#pragma unroll
    for (int v = 0; v < V; ++v) u[v] += xor3(s0[v], w[v], j0[v]) + xor3(s1[v], w[v], j1[v]);
    lds_load_n<V>(s0, sp + (pu << lgPl) + (y << lgG) + g0);    // plane z-1
    lds_load_n<V>(s1, sp + (pd << lgPl) + (y << lgG) + g0);    // plane z+1
    lds_load_n<V>(j0, bz + (pu << lgPl) + (y << lgG) + g0);
    lds_load_n<V>(j1, bz + rowb + g0);
#pragma unroll
    for (int v = 0; v < V; ++v) u[v] += xor3(s0[v], w[v], j0[v]) + xor3(s1[v], w[v], j1[v]);
  }
  const uint8_t *tb = reinterpret_cast<const uint8_t *>(thr);
#pragma unroll
  for (int v = 0; v < V; ++v) nw[v] = decide_n<WIDE>(w[v], u[v], off, r[v], tb, t);
  lds_store_n<V>(sp + rowb + g0, nw);
}

// One workgroup of the 2D tiled sweep: tile `tile` of walker `w`, staged in
// sp (LDS), k sweeps, interior written back; per-sweep tallies to acc3.
// s_sw != NULL (whole replicas, one workgroup per walker): the per-sweep
// tallies go there instead.
template <int V>
__device__ __forceinline__ void tiled_n_body(const TiledArgs &a, uint32_t tile, uint32_t w,
                                             uint32_t *sp, uint64_t *s_thr,
                                             int (*s_red)[2], int (*s_sw)[2] = nullptr) {
  const Geometry &G = a.geo;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t L = G.L, lgL = a.lg_L, lgG = lgL - 3u, gmask = (1u << lgG) - 1u;
  const uint32_t y0 = tile * a.H;
  const uint32_t Ht = min(a.H, L - y0);
  const uint32_t halo = a.halo;
  const uint32_t np = Ht + 2u * halo;                  // LDS rows
  const uint32_t base = (y0 + L - halo) & (L - 1u);   // global row of LDS row 0
  const uint32_t slot = a.st.slot_of[w];
  if (tid < kClasses) s_thr[tid] = a.st.flip_cmp[slot * kClasses + tid];

  // rows [base, base+np) mod L of this walker, four bits per site; a packed
  // word (32 sites) becomes four LDS dwords (rows shorter than a word only
  // occur in whole-replica tiles, which start at row 0)
  const uint32_t nwr = G.N >> 5;
  unpack_tile_n(sp, a.src + (size_t)w * nwr, (base * L) >> 5, (np * L) >> 5, nwr - 1u, tid, nt);
  __syncthreads();

  const uint32_t smask = (1u << a.lg_spr) - 1u;
  TallyN t = {0u, 0u, 0u};
  for (uint32_t hs = 0; hs < 2u * a.sch.nsw; ++hs) {
    const uint32_t c = hs & 1u;
    const uint32_t s = a.sch.s0 + (hs >> 1);
    const uint32_t ext = halo ? (halo - 1u - hs) : 0u;
    const uint32_t plo = halo - ext;                 // computed LDS rows [plo, plo+Ht+2ext)
    // wrap: rows 0 and np-1 have their neighbours across the tile (whole-replica tiles only)
    auto item = [&](auto vtag, auto wrap, uint32_t pl, uint32_t g0, bool interior) {
      constexpr int VV = decltype(vtag)::value;
      const uint32_t pu = (decltype(wrap)::value && pl == 0u) ? np - 1u : pl - 1u;
      const uint32_t pd = (decltype(wrap)::value && pl + 1u == np) ? 0u : pl + 1u;
      const uint32_t gp = (base + pl) & (L - 1u);   // global row
      const uint32_t off = (c + gp) & 1u;
      const uint32_t ctr0 = (gp << lgG) + g0;
      Words r[VV];
#pragma unroll
      for (int v = 0; v < VV; ++v)
        r[v] = philox(ctr0 + v, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
      TallyN tg = {0u, 0u, 0u};
      span2d_n<VV>(sp + (pl << lgG), sp + (pu << lgG), sp + (pd << lgG), g0, gmask, off, r, s_thr, tg);
      if (interior) {
        t.n += tg.n;
        t.sb += tg.sb;
        t.sc += tg.sc;
      }
    };
    if (halo) {
      // interior rows as V-dword spans, the 2 ext recomputed halo rows as
      // single dwords spread over every lane
      const uint32_t items = Ht << a.lg_spr;
      for (uint32_t q = tid; q < items; q += nt)
        item(std::integral_constant<int, V>{}, std::false_type{}, halo + (q >> a.lg_spr),
             (q & smask) * V, true);
      const uint32_t hitems = (2u * ext) << lgG;
      for (uint32_t q = tid; q < hitems; q += nt) {
        const uint32_t r = q >> lgG;
        const uint32_t pl = r < ext ? plo + r : halo + Ht + (r - ext);
        item(std::integral_constant<int, 1>{}, std::false_type{}, pl, q & gmask, false);
      }
    } else {
      const uint32_t items = Ht << a.lg_spr;
      for (uint32_t q = tid; q < items; q += nt)
        item(std::integral_constant<int, V>{}, std::true_type{}, q >> a.lg_spr, (q & smask) * V,
             true);
    }
    if (c == 1u) {
      // per flip: dE_int = 2z - 4u, dM = 4b - 2
      int dE = a.z2 * (int)t.n - 4 * ((int)t.sc - 8 * (int)t.sb);
      int dM = 4 * (int)t.sb - 2 * (int)t.n;
      t = {0u, 0u, 0u};
      dE = wave_total(dE);
      dM = wave_total(dM);
      if ((tid & 63u) == 0u) {
        s_red[tid >> 6][0] = dE;
        s_red[tid >> 6][1] = dM;
      }
    }
    __syncthreads();
    if (c == 1u && tid == 0u) {
      int sE = 0, sM = 0;
      for (uint32_t v = 0; v < (nt >> 6); ++v) {
        sE += s_red[v][0];
        sM += s_red[v][1];
      }
      if (s_sw) {
        s_sw[hs >> 1][0] = sE;
        s_sw[hs >> 1][1] = sM;
      } else {
        int32_t *acc = a.st.acc3 + ((size_t)(hs >> 1) * G.R + w) * 4u;
        __hip_atomic_fetch_add(acc, sE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(acc + 1, sM, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }

  // interior rows back to HBM, packed (contiguous)
  pack_tile_n(a.dst + (size_t)w * nwr + ((y0 * L) >> 5), sp + ((size_t)halo << lgG), (Ht * L) >> 5,
              tid, nt);
}

template <int V>
__global__ __launch_bounds__(kMaxThreads) void k_tiled_n(TiledArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint64_t s_thr[kClasses];
  __shared__ int s_red[kMaxThreads / 64][2];
  __shared__ int s_sw[kMaxSweepsPerLaunch][2];
  __shared__ uint32_t s_last;
  const bool whole = a.halo == 0u; // whole replicas: one workgroup per walker
  tiled_n_body<V>(a, blockIdx.x, blockIdx.y, reinterpret_cast<uint32_t *>(smem), s_thr, s_red,
                  whole ? s_sw : nullptr);
  // whole replicas fold themselves and leave the exchange step to a launch of
  // its own (launch_tiled): no arrival counter for a last workgroup
  if (whole) {
    if (threadIdx.x == 0u) fold_own_walker(a, blockIdx.y, s_sw);
  } else {
    tiled_epilogue(a, threadIdx.x, blockDim.x, &s_last, gridDim.x * gridDim.y);
  }
}


// Batched 2D tiled sweep: the tiled kernel's work for many instances of one
// lattice size in one launch.  Each instance's schedule (sweep, records,
// exchange step, spin buffer) comes from its device counters; its last
// workgroup to finish (its own arrival counter) runs its epilogue.
template <int V>
__global__ __launch_bounds__(kMaxThreads) void k_batch_tiled(const BatchInst *insts,
                                                             const BatchTileItem *items,
                                                             uint32_t H, uint32_t K) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint64_t s_thr[kClasses];
  __shared__ int s_red[kMaxThreads / 64][2];
  __shared__ uint32_t s_last;
  const BatchTileItem it = items[blockIdx.x];
  const BatchInst &I = insts[it.inst];
  const uint32_t nsw = cycle_sweeps(I.ctr, K);
  if (nsw == 0u) return; // every workgroup of an idle instance leaves here
  const uint32_t tiles = I.ctr[kCtrTiles], every = I.ctr[kCtrEvery], cur = I.ctr[kCtrCur];
  TiledArgs a;
  a.st = I.st;
  a.geo = I.geo;
  a.key = I.key;
  a.sch.s0 = I.ctr[kCtrSweeps];
  a.sch.nsw = nsw;
  a.sch.record_every = I.record_every;
  a.sch.rec_base = I.ctr[kCtrRecords];
  a.sch.exchange_every = every;
  a.sch.do_exchange = (every && (a.sch.s0 + nsw) % every == 0u) ? 1u : 0u;
  a.sch.ex_step = I.ctr[kCtrExchanges];
  a.H = H;
  a.halo = tiles > 1u ? 2u * nsw : 0u;
  a.src = I.st.spins[cur];
  a.dst = a.halo ? I.st.spins[cur ^ 1u] : I.st.spins[cur];
  a.lg_L = I.lg_L;
  a.lg_spr = I.lg_L - 3u - (V == 8 ? 3u : V == 4 ? 2u : V == 2 ? 1u : 0u);
  a.lg_rows = 0u;
  a.z2 = I.z2;
  tiled_n_body<V>(a, it.tile, it.w, reinterpret_cast<uint32_t *>(smem), s_thr, s_red);
  tiled_epilogue(a, threadIdx.x, blockDim.x, &s_last, I.geo.R * max(tiles, 1u));
}

// 3D +-J EA tiled sweep (nibble layout): tiles of z-planes with halo planes.
template <int DIM, int V>
__global__ __launch_bounds__(kMaxThreads) void k_tiled(TiledArgs a) {
  static_assert(DIM == 3, "2D lattices use k_tiled_n");
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint64_t s_thr[kClasses];
  __shared__ int s_red[kMaxThreads / 64][2];
  __shared__ uint32_t s_last;

  const Geometry &G = a.geo;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t tile = blockIdx.x, w = blockIdx.y;
  const uint32_t L = G.L, lgL = a.lg_L;
  const uint32_t lgG = lgL - 3u, gmask = (1u << lgG) - 1u;   // dwords per row
  const uint32_t lgPl = lgL + lgG;                           // dwords per plane
  const uint32_t y0 = tile * a.H;
  const uint32_t Ht = min(a.H, L - y0);
  const uint32_t halo = a.halo;
  const uint32_t np = Ht + 2u * halo;                  // LDS planes
  const uint32_t base = (y0 + L - halo) & (L - 1u);   // global plane of LDS plane 0
  const uint32_t slot = a.st.slot_of[w];
  if (tid < kClasses) s_thr[tid] = a.st.flip_cmp[slot * kClasses + tid];

  // four bits per site: spins, then the x, y, z bond planes of the tile
  uint32_t *sp = reinterpret_cast<uint32_t *>(smem);
  uint32_t *bx = sp + ((size_t)np << lgPl);
  uint32_t *by = bx + ((size_t)np << lgPl);
  uint32_t *bz = by + ((size_t)np << lgPl);

  // Stage planes [base, base+np) mod L of this walker and of the bonds.
  {
    const uint32_t nwr = G.N >> 5, wpp = (L * L) >> 5;  // packed words per plane
    const uint32_t first = base * wpp, cnt = np * wpp;
    unpack_tile_n(sp, a.src + (size_t)w * nwr, first, cnt, nwr - 1u, tid, nt);
    unpack_tile_n(bx, a.st.bonds, first, cnt, nwr - 1u, tid, nt);
    unpack_tile_n(by, a.st.bonds + nwr, first, cnt, nwr - 1u, tid, nt);
    unpack_tile_n(bz, a.st.bonds + 2u * nwr, first, cnt, nwr - 1u, tid, nt);
  }
  __syncthreads();

  const uint32_t smask = (1u << a.lg_spr) - 1u, rmask = G.rows - 1u;
  const uint32_t shp = a.lg_spr + a.lg_rows;
  TallyN t = {0u, 0u, 0u};
  for (uint32_t hs = 0; hs < 2u * a.sch.nsw; ++hs) {
    const uint32_t c = hs & 1u;
    const uint32_t s = a.sch.s0 + (hs >> 1);
    const uint32_t ext = halo ? (halo - 1u - hs) : 0u;
    const uint32_t plo = halo - ext;                 // computed LDS planes [plo, plo+Ht+2ext)
    const uint32_t items = (Ht + 2u * ext) << shp;
    for (uint32_t q = tid; q < items; q += nt) {
      const uint32_t pl = plo + (q >> shp);
      const uint32_t y = (q >> a.lg_spr) & rmask;
      const uint32_t g0 = (q & smask) * V;
      const uint32_t pu = (pl == 0u) ? np - 1u : pl - 1u;
      const uint32_t pd = (pl + 1u == np) ? 0u : pl + 1u;
      const uint32_t gp = (base + pl) & (L - 1u);   // global plane coordinate
      const uint32_t off = (c + gp + y) & 1u;
      const uint32_t ctr0 = (((gp << a.lg_rows) + y) << lgG) + g0;
      Words r[V];
#pragma unroll
      for (int v = 0; v < V; ++v)
        r[v] = philox(ctr0 + v, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
      TallyN tg = {0u, 0u, 0u};
      span3d_n<V>(sp, bx, by, bz, lgG, lgPl, pl, pu, pd, y, (y + L - 1u) & (L - 1u),
                  (y + 1u) & (L - 1u), g0, gmask, off, r, s_thr, tg);
      if (pl >= halo && pl < halo + Ht) {
        t.n += tg.n;
        t.sb += tg.sb;
        t.sc += tg.sc;
      }
    }
    if (c == 1u) {
      int dE = a.z2 * (int)t.n - 4 * ((int)t.sc - 8 * (int)t.sb);
      int dM = 4 * (int)t.sb - 2 * (int)t.n;
      t = {0u, 0u, 0u};
      dE = wave_total(dE);
      dM = wave_total(dM);
      if ((tid & 63u) == 0u) {
        s_red[tid >> 6][0] = dE;
        s_red[tid >> 6][1] = dM;
      }
    }
    __syncthreads();
    if (c == 1u && tid == 0u) {
      int sE = 0, sM = 0;
      for (uint32_t v = 0; v < (nt >> 6); ++v) {
        sE += s_red[v][0];
        sM += s_red[v][1];
      }
      int32_t *acc = a.st.acc3 + ((size_t)(hs >> 1) * G.R + w) * 4u;
      __hip_atomic_fetch_add(acc, sE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(acc + 1, sM, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }

  // Write the interior planes back, packed (contiguous in global memory).
  pack_tile_n(a.dst + (size_t)w * (G.N >> 5) + y0 * ((L * L) >> 5), sp + ((size_t)halo << lgPl),
              Ht * ((L * L) >> 5), tid, nt);
  tiled_epilogue(a, tid, nt, &s_last, gridDim.x * gridDim.y);
}

// ---- rows that are not whole 8-site groups (2D, any even L) ----------------
// When 8 does not divide L (or L is not a power of two), the site groups that
// share a Philox block -- sites 8G .. 8G+7 of the walker in site order -- do not
// line up with the rows.  Row y then starts at nibble ph = (y L) mod 8 of group
// G0 = floor(y L / 8), and the LDS keeps each row as its own run of dwords
// "phased" like that: dword g of row y holds group G0 + g, nibble n the site
// x = 8 g + n - ph when 0 <= x < L (other nibbles are padding, never flipped).
// Every dword is then still exactly one Philox group, and the checkerboard
// colour of nibble n is (n + y) mod 2 as before.  The row above or below has
// another phase ph': its sites appear shifted by d = ph' - ph nibbles, which a
// funnel shift (v_alignbit) of two adjacent dwords of that row undoes.  Inside
// a row the left and right neighbours are the adjacent nibbles, except at the
// periodic wrap: the first and last dwords of a row are single-group items that
// patch x = 0's left neighbour (x = L-1) and x = L-1's right neighbour (x = 0),
// and mask their padding nibbles out of the decision.  The whole replica stays
// in LDS for the launch (in place).
constexpr uint32_t kPhasedLead = 3u; // LDS dword of row 0's group 0, so that group 1 is 16-byte aligned

struct PhasedArgs {
  TiledArgs t;   // H = L, halo = 0: whole replicas, updated in place
  uint32_t S;    // LDS dwords per row (a multiple of 4)
  uint32_t Gmax; // groups a row touches, at most
  uint32_t nI;   // interior spans per row: groups 1 + V k .. 1 + V k + V - 1, k < nI
  uint32_t nE;   // single-group items per row: group 0, then groups 1 + V nI .. Gmax - 1
  uint32_t lds_rows; // LDS dword of the per-row table
};

// Nibbles [lo, hi) of a dword, 0 <= lo <= hi <= 8, as the low bit of each nibble.
__device__ __forceinline__ uint32_t nibble_bits(uint32_t lo, uint32_t hi) {
  const uint32_t a = hi >= 8u ? 0xFFFFFFFFu : (1u << (4u * hi)) - 1u;
  const uint32_t b = lo >= 8u ? 0xFFFFFFFFu : (1u << (4u * lo)) - 1u;
  return (a & ~b) & 0x11111111u;
}

// Per-row constants, one uint4 per row in LDS: x = first group G0, y = LDS
// dword of group 0 | shift of the row above << 16 | shift of the row below
// << 21 | phase << 26, z / w = LDS dword of the first of the two dwords whose
// funnel shift gives the view of the row above / below at group 0.
__device__ __forceinline__ uint4 phased_row_info(uint32_t y, uint32_t L, uint32_t S) {
  const uint32_t yu = y ? y - 1u : L - 1u, yd = (y + 1u == L) ? 0u : y + 1u;
  const uint32_t ph = (y * L) & 7u, phu = (yu * L) & 7u, phd = (yd * L) & 7u;
  const int du = (int)phu - (int)ph, dd = (int)phd - (int)ph;
  const uint32_t base = kPhasedLead + y * S;
  const uint32_t bu = kPhasedLead + yu * S - (du < 0 ? 1u : 0u);
  const uint32_t bd = kPhasedLead + yd * S - (dd < 0 ? 1u : 0u);
  const uint32_t shu = (uint32_t)(4 * du) & 31u, shd = (uint32_t)(4 * dd) & 31u;
  return make_uint4((y * L) >> 3, base | (shu << 16) | (shd << 21) | (ph << 26), bu, bd);
}

// Interior span: V full dwords g0 .. g0+V-1 (1 <= g0, g0+V < the row's last dword)
// of the row at LDS dword `base`; vu, vd = first dwords of the V+1 dwords of the
// rows above and below whose funnel shifts by shu, shd align them with this row.
template <int V>
__device__ __forceinline__ void span_phased(uint32_t *lds, uint32_t base, uint32_t g0, uint32_t vu,
                                            uint32_t shu, uint32_t vd, uint32_t shd, uint32_t off,
                                            const Words (&r)[V], const uint64_t *thr, TallyN &t) {
  uint32_t *row = lds + base;
  uint32_t w[V], a[V + 1], b[V + 1], nw[V];
  lds_load_n<V>(w, row + g0);
#pragma unroll
  for (int i = 0; i <= V; ++i) {
    a[i] = lds[vu + g0 + i];
    b[i] = lds[vd + g0 + i];
  }
  // the neighbouring dword on the side the colour sites need (as in span2d_n)
  const uint32_t e = row[off ? g0 + V : g0 - 1u];
  const uint8_t *tb = reinterpret_cast<const uint8_t *>(thr);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint32_t l = __builtin_amdgcn_alignbit(w[v], v ? w[v - 1] : e, 28u);
    const uint32_t rr = __builtin_amdgcn_alignbit(v < V - 1 ? w[v + 1] : e, w[v], 4u);
    const uint32_t up = __builtin_amdgcn_alignbit(a[v + 1], a[v], shu);
    const uint32_t dn = __builtin_amdgcn_alignbit(b[v + 1], b[v], shd);
    uint32_t u = rr ^ w[v];
    u = xad(l, w[v], u);
    u = xad(dn, w[v], u);
    u = xad(up, w[v], u);
    nw[v] = decide_n<true>(w[v], u, off, r[v], tb, t);
  }
  lds_store_n<V>(row + g0, nw);
}

// Edge item: the single dword g of a row of phase ph (its first or last dwords):
// padding nibbles masked out of the decision, the row's periodic wrap patched in.
__device__ __forceinline__ void edge_phased(uint32_t *lds, uint32_t base, uint32_t g, uint32_t ph,
                                            uint32_t L, uint32_t vu, uint32_t shu, uint32_t vd,
                                            uint32_t shd, uint32_t off, const Words &r,
                                            const uint64_t *thr, TallyN &t) {
  uint32_t *row = lds + base;
  const uint32_t w = row[g];
  uint32_t l = __builtin_amdgcn_alignbit(w, row[(int)g - 1], 28); // g = 0: the dword before the row
  uint32_t rr = __builtin_amdgcn_alignbit(row[g + 1u], w, 4u);
  // sites of the row occupy nibbles ph .. ph + L - 1 counted from group 0
  const int lo = (int)ph - 8 * (int)g, hi = (int)(ph + L) - 8 * (int)g;
  const uint32_t vm = nibble_bits((uint32_t)min(max(lo, 0), 8), (uint32_t)min(max(hi, 0), 8));
  if (lo >= 0 && lo < 8) { // x = 0 sits here: its left neighbour is x = L - 1
    const uint32_t pl = ph + L - 1u;
    const uint32_t xv = (row[pl >> 3] >> (4u * (pl & 7u))) & 0xFu;
    const uint32_t sh = 4u * (uint32_t)lo;
    l = (l & ~(0xFu << sh)) | (xv << sh);
  }
  if (hi >= 1 && hi <= 8) { // x = L - 1 sits here: its right neighbour is x = 0
    const uint32_t xv = (row[ph >> 3] >> (4u * (ph & 7u))) & 0xFu;
    const uint32_t sh = 4u * (uint32_t)(hi - 1);
    rr = (rr & ~(0xFu << sh)) | (xv << sh);
  }
  const uint32_t up = __builtin_amdgcn_alignbit(lds[vu + g + 1u], lds[vu + g], shu);
  const uint32_t dn = __builtin_amdgcn_alignbit(lds[vd + g + 1u], lds[vd + g], shd);
  uint32_t u = rr ^ w;
  u = xad(l, w, u);
  u = xad(dn, w, u);
  u = xad(up, w, u);
  // decide_n with the padding nibbles excluded: a nibble flips only if it is a site
  const uint32_t M = off ? 0xF0F0F0F0u : 0x0F0F0F0Fu;
  const uint32_t rot = off ? 1u : 29u;
  const uint32_t cls = ((w << 3) | u) & M;
  const uint32_t c8 = __builtin_amdgcn_alignbit(cls, cls, rot);
  const uint8_t *tb = reinterpret_cast<const uint8_t *>(thr);
  const uint64_t t0 = *reinterpret_cast<const uint64_t *>(tb + (c8 & 0xFFu));
  const uint64_t t1 = *reinterpret_cast<const uint64_t *>(tb + __builtin_amdgcn_ubfe(c8, 8u, 8u));
  const uint64_t t2 = *reinterpret_cast<const uint64_t *>(tb + __builtin_amdgcn_ubfe(c8, 16u, 8u));
  const uint64_t t3 = *reinterpret_cast<const uint64_t *>(tb + (c8 >> 24));
  const uint32_t a01 = __builtin_amdgcn_perm(carry_mask(r.y, t1), carry_mask(r.x, t0), 0x0C0C0400u);
  const uint32_t a23 = __builtin_amdgcn_perm(carry_mask(r.w, t3), carry_mask(r.z, t2), 0x04000C0Cu);
  const uint32_t f = __builtin_amdgcn_bitop3_b32(a01, a23, 0x01010101u << (4u * off), 0xA8) & vm;
  t.n += __builtin_popcount(f);
  t.sb = __builtin_amdgcn_udot8(w, f, t.sb, false);
  t.sc = __builtin_amdgcn_udot8(cls, f, t.sc, false);
  row[g] = w ^ f;
}

// Edge item of a row whose two ends lie in different dwords (at least two
// groups per row): dword g is the row's first (g = 0, x = 0 at nibble ph), one
// between the interior spans and the last (all nibbles sites), the last (g =
// pl >> 3 with pl = ph + L - 1, x = L - 1 at nibble pl & 7) or past it (all
// padding).  The periodic wrap is one nibble patched into the left view of the
// first dword or the right view of the last; padding nibbles are masked out
// of the decision.  The same instructions serve every kind, selected per lane.
__device__ __forceinline__ void edge_phased_2(uint32_t *lds, uint32_t base, uint32_t g, uint32_t ph,
                                              uint32_t pl, uint32_t vu, uint32_t shu, uint32_t vd,
                                              uint32_t shd, uint32_t off, const Words &r,
                                              const uint64_t *thr, TallyN &t) {
  uint32_t *row = lds + base;
  const uint32_t w = row[g];
  uint32_t l = __builtin_amdgcn_alignbit(w, row[(int)g - 1], 28u); // g = 0: the dword before the row
  uint32_t rr = __builtin_amdgcn_alignbit(row[g + 1u], w, 4u);
  const uint32_t gl = pl >> 3;
  const bool first = g == 0u, last = g == gl;
  // x = 0's left neighbour is x = L - 1 (nibble pl), x = L - 1's right one x = 0 (nibble ph)
  const uint32_t src = first ? pl : ph;
  const uint32_t xv = (row[src >> 3] >> (4u * (src & 7u))) & 0xFu;
  const uint32_t sh = 4u * (first ? ph : (pl & 7u));
  const uint32_t pm = (first || last) ? (0xFu << sh) : 0u;
  const uint32_t x = (pm & (xv << sh)) | (~pm & (first ? l : rr));
  l = first ? x : l;
  rr = first ? rr : x;
  const uint32_t vm = first ? (0x11111111u << (4u * ph))
                    : g < gl ? 0x11111111u
                    : last   ? (0x11111111u >> (28u - 4u * (pl & 7u)))
                             : 0u;
  const uint32_t up = __builtin_amdgcn_alignbit(lds[vu + g + 1u], lds[vu + g], shu);
  const uint32_t dn = __builtin_amdgcn_alignbit(lds[vd + g + 1u], lds[vd + g], shd);
  uint32_t u = rr ^ w;
  u = xad(l, w, u);
  u = xad(dn, w, u);
  u = xad(up, w, u);
  row[g] = decide_n<true>(w, u, off, r, reinterpret_cast<const uint8_t *>(thr), t, vm);
}

// The first and last dwords of a row whose ends lie in different dwords, as
// one item: x = 0 (nibble ph of dword 0) and x = L - 1 (nibble pl & 7 of dword
// gl = pl >> 3) are each other's periodic neighbours, so each patches the
// other's view straight from registers.
__device__ __forceinline__ void edge_pair_phased(uint32_t *lds, uint32_t base, uint32_t gl,
                                                 uint32_t ph, uint32_t pl, uint32_t vu, uint32_t shu,
                                                 uint32_t vd, uint32_t shd, uint32_t off,
                                                 const Words &r0, const Words &rl,
                                                 const uint64_t *thr, TallyN &t) {
  uint32_t *row = lds + base;
  const uint32_t w0 = row[0], wl = row[gl];
  uint32_t l0 = __builtin_amdgcn_alignbit(w0, row[-1], 28u); // the dword before the row: padding
  const uint32_t r0v = __builtin_amdgcn_alignbit(row[1], w0, 4u);
  const uint32_t ll = __builtin_amdgcn_alignbit(wl, row[gl - 1u], 28u);
  uint32_t rlv = __builtin_amdgcn_alignbit(row[gl + 1u], wl, 4u);
  const uint32_t s0 = 4u * ph, sl = 4u * (pl & 7u);
  l0 = (l0 & ~(0xFu << s0)) | (((wl >> sl) & 0xFu) << s0);
  rlv = (rlv & ~(0xFu << sl)) | (((w0 >> s0) & 0xFu) << sl);
  const uint32_t up0 = __builtin_amdgcn_alignbit(lds[vu + 1u], lds[vu], shu);
  const uint32_t dn0 = __builtin_amdgcn_alignbit(lds[vd + 1u], lds[vd], shd);
  const uint32_t upl = __builtin_amdgcn_alignbit(lds[vu + gl + 1u], lds[vu + gl], shu);
  const uint32_t dnl = __builtin_amdgcn_alignbit(lds[vd + gl + 1u], lds[vd + gl], shd);
  uint32_t u0 = r0v ^ w0;
  u0 = xad(l0, w0, u0);
  u0 = xad(dn0, w0, u0);
  u0 = xad(up0, w0, u0);
  uint32_t ul = rlv ^ wl;
  ul = xad(ll, wl, ul);
  ul = xad(dnl, wl, ul);
  ul = xad(upl, wl, ul);
  const uint8_t *tb = reinterpret_cast<const uint8_t *>(thr);
  row[0] = decide_n<true>(w0, u0, off, r0, tb, t, 0x11111111u << s0);
  row[gl] = decide_n<true>(wl, ul, off, rl, tb, t, 0x11111111u >> (28u - sl));
}

// Whole-replica sweep of phased rows: grid (1, R), one workgroup per walker.
template <int V>
__global__ __launch_bounds__(kMaxThreads) void k_phased(PhasedArgs pa) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint64_t s_thr[kClasses];
  __shared__ int s_red[kMaxThreads / 64][2];
  __shared__ int s_sw[kMaxSweepsPerLaunch][2]; // this walker's dE, dM per sweep
  const TiledArgs &a = pa.t;
  const Geometry &G = a.geo;
  const uint32_t tid = threadIdx.x, nt = blockDim.x, w = blockIdx.y;
  const uint32_t L = G.L, S = pa.S, nwr = G.nwr;
  uint32_t *lds = reinterpret_cast<uint32_t *>(smem);
  uint4 *rows = reinterpret_cast<uint4 *>(lds + pa.lds_rows);
  const uint32_t slot = a.st.slot_of[w];
  if (tid < kClasses) s_thr[tid] = a.st.flip_cmp[slot * kClasses + tid];

  // stage: LDS dword (y, g) <- byte G0(y) + g of the walker's packed sites
  // (one byte = one group of 8 sites), every other nibble zero.
  if constexpr (V > 1) {
    // At least 6 groups per row: a group's sites lie in at most two rows.
    // Packed words are loaded whole, all of a thread's loads issued together
    // (one memory round trip), and each group's byte is spread to the row of
    // its first site and, when it runs past that row's end, to dword 0 of the
    // next row; the dwords past a row's last group, and those around the
    // rows, are zeroed (no stencil may carry out of a padding nibble).
    const uint32_t *src = a.src + (size_t)w * nwr;
    const uint32_t N = G.N;
    const float invL = 1.0f / (float)L;
    constexpr uint32_t kBatch = 8;
    for (uint32_t q0 = tid; q0 < nwr; q0 += kBatch * nt) {
      uint32_t v[kBatch];
#pragma unroll
      for (uint32_t j = 0; j < kBatch; ++j) v[j] = q0 + j * nt < nwr ? src[q0 + j * nt] : 0u;
#pragma unroll
      for (uint32_t j = 0; j < kBatch; ++j) {
        const uint32_t q = q0 + j * nt;
        if (q >= nwr) break;
#pragma unroll
        for (uint32_t b = 0; b < 4u; ++b) {
          const uint32_t gi = 4u * q + b, x0 = 8u * gi; // the group's first site
          if (x0 >= N) break;
          uint32_t y = (uint32_t)((float)x0 * invL); // within one of the row index
          y -= y * L > x0 ? 1u : 0u;
          y += (y + 1u) * L <= x0 ? 1u : 0u;
          const uint32_t val = spread8((v[j] >> (8u * b)) & 0xFFu);
          lds[kPhasedLead + y * S + (gi - ((y * L) >> 3))] = val;
          if (x0 + 8u > (y + 1u) * L && y + 1u < L) lds[kPhasedLead + (y + 1u) * S] = val;
        }
      }
    }
    for (uint32_t y = tid; y < L; y += nt) {
      const uint32_t gl = (((y * L) & 7u) + L - 1u) >> 3; // the row's last group
      for (uint32_t g = gl + 1u; g < S; ++g) lds[kPhasedLead + y * S + g] = 0u;
      rows[y] = phased_row_info(y, L, S);
    }
    if (tid < kPhasedLead) lds[tid] = 0u;
    if (tid < 4u) lds[kPhasedLead + L * S + tid] = 0u;
  } else {
    // Each thread steps through (y, g) by nt dwords at a time (no divisions
    // in the loop) and issues four loads before it spreads any of them.
    const uint8_t *src = reinterpret_cast<const uint8_t *>(a.src + (size_t)w * nwr);
    const uint32_t nbytes = 4u * nwr, Gmax = pa.Gmax;
    if (tid < kPhasedLead) lds[tid] = 0u;
    if (tid < 4u) lds[kPhasedLead + L * S + tid] = 0u;
    const uint32_t sy = nt / S, sg = nt - sy * S;
    uint32_t y = tid / S, g = tid - y * S;
    while (y < L) {
      constexpr int kBatch = 4;
      uint32_t q[kBatch], b[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const uint32_t byte = ((y * L) >> 3) + g;
        q[j] = y < L ? kPhasedLead + y * S + g : 0xFFFFFFFFu;
        b[j] = (y < L && g < Gmax && byte < nbytes) ? src[byte] : 0u;
        g += sg;
        y += sy;
        if (g >= S) {
          g -= S;
          ++y;
        }
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j)
        if (q[j] != 0xFFFFFFFFu) lds[q[j]] = spread8(b[j]);
    }
    for (uint32_t yy = tid; yy < L; yy += nt) rows[yy] = phased_row_info(yy, L, S);
  }
  __syncthreads();

  // each thread's first items, stepped by nt items per round without divisions
  const uint32_t nI = pa.nI;
  // edge items per row: with at least 6 groups per row (V > 1) the row's first
  // and last dwords are one item, the other edge dwords one item each
  const uint32_t nE = V > 1 ? pa.nE - 1u : pa.nE;
  const uint32_t iy0 = nI ? tid / nI : L, ik0 = nI ? tid - iy0 * nI : 0u; // no interior spans: skip
  const uint32_t idy = nI ? nt / nI : 0u, idk = nI ? nt - idy * nI : 0u;
  const uint32_t ey0 = tid / nE, ek0 = tid - ey0 * nE;
  const uint32_t edy = nt / nE, edk = nt - edy * nE;
  TallyN t = {0u, 0u, 0u};
  for (uint32_t hs = 0; hs < 2u * a.sch.nsw; ++hs) {
    const uint32_t c = hs & 1u;
    const uint32_t s = a.sch.s0 + (hs >> 1);
    // interior spans
    for (uint32_t y = iy0, k = ik0; y < L;) {
      const uint4 ri = rows[y];
      const uint32_t base = ri.y & 0xFFFFu, shu = (ri.y >> 16) & 31u, shd = (ri.y >> 21) & 31u;
      const uint32_t g0 = 1u + k * V, off = (c + y) & 1u;
      Words r[V];
#pragma unroll
      for (int v = 0; v < V; ++v)
        r[v] = philox(ri.x + g0 + v, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
      span_phased<V>(lds, base, g0, ri.z, shu, ri.w, shd, off, r, s_thr, t);
      k += idk;
      y += idy;
      if (k >= nI) {
        k -= nI;
        ++y;
      }
    }
    // first and last dwords of every row
    for (uint32_t y = ey0, k = ek0; y < L;) {
      const uint4 ri = rows[y];
      const uint32_t base = ri.y & 0xFFFFu, shu = (ri.y >> 16) & 31u, shd = (ri.y >> 21) & 31u;
      const uint32_t ph = ri.y >> 26, off = (c + y) & 1u;
      if constexpr (V > 1) {
        // at least 6 groups per row: the two ends lie in different dwords
        const uint32_t pl = ph + L - 1u, gl = pl >> 3;
        if (k == 0u) {
          const Words r0 = philox(ri.x, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
          const Words rl = philox(ri.x + gl, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
          edge_pair_phased(lds, base, gl, ph, pl, ri.z, shu, ri.w, shd, off, r0, rl, s_thr, t);
        } else {
          uint32_t g = nI * V + k; // the other edge dwords, the last one skipped
          g += g >= gl ? 1u : 0u;
          const Words r = philox(ri.x + g, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
          edge_phased_2(lds, base, g, ph, pl, ri.z, shu, ri.w, shd, off, r, s_thr, t);
        }
      } else {
        const uint32_t g = k ? nI * V + k : 0u;
        const Words r = philox(ri.x + g, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
        edge_phased(lds, base, g, ph, L, ri.z, shu, ri.w, shd, off, r, s_thr, t);
      }
      k += edk;
      y += edy;
      if (k >= nE) {
        k -= nE;
        ++y;
      }
    }
    if (c == 1u) {
      // per flip: dE_int = 2z - 4u, dM = 4b - 2
      int dE = a.z2 * (int)t.n - 4 * ((int)t.sc - 8 * (int)t.sb);
      int dM = 4 * (int)t.sb - 2 * (int)t.n;
      t = {0u, 0u, 0u};
      dE = wave_total(dE);
      dM = wave_total(dM);
      if ((tid & 63u) == 0u) {
        s_red[tid >> 6][0] = dE;
        s_red[tid >> 6][1] = dM;
      }
    }
    __syncthreads();
    if (c == 1u && tid == 0u) {
      int sE = 0, sM = 0;
      for (uint32_t v = 0; v < (nt >> 6); ++v) {
        sE += s_red[v][0];
        sM += s_red[v][1];
      }
      s_sw[hs >> 1][0] = sE;
      s_sw[hs >> 1][1] = sM;
    }
  }

  if (tid == 0u) fold_own_walker(a, w, s_sw);

  // back to HBM: packed word q holds groups 4q .. 4q+3; a group's sites lie in
  // the row of its first site and, past that row's end, in the next row's group 0
  {
    uint32_t *dst = a.dst + (size_t)w * nwr;
    const uint32_t N = G.N;
    for (uint32_t q = tid; q < nwr; q += nt) {
      uint32_t word = 0u;
      uint32_t y = (32u * q) / L;
#pragma unroll
      for (uint32_t b = 0; b < 4u; ++b) {
        const uint32_t i0 = 32u * q + 8u * b; // first site of the group
        if (i0 >= N) break;
        while (i0 >= (y + 1u) * L) ++y;
        const uint32_t G0 = (y * L) >> 3, gi = 4u * q + b;
        const uint32_t k = min(8u, (y + 1u) * L - i0); // sites of the group in row y
        uint32_t bits = lds[kPhasedLead + y * S + (gi - G0)] & nibble_bits(0u, k);
        if (k < 8u && y + 1u < L) bits |= lds[kPhasedLead + (y + 1u) * S] & nibble_bits(k, 8u);
        word |= gather8(bits) << (8u * b);
      }
      dst[q] = word;
    }
  }
  // the exchange step, if any, is the next launch's (launch_tiled)
}

struct FusedArgs {
  DevState st;
  Geometry geo;
  Keys key;
  Schedule sch;
  uint32_t *spins; // bit-packed, updated in place
  uint32_t lg_L, lg_spr, lg_rows, lg_items; // log2 of L, spans per row, rows per plane, spans per replica
  int32_t z2;
  uint32_t ntab; // swap-table entries staged in LDS (0: the rows are read from device memory)
};

// LDS layout of the fused kernel: thresholds, maps, E and M, the swap test's
// per-pair data and counters, optionally the swap-table rows, the lattices.
struct FusedLayout {
  uint32_t thr, wat, sof, E, M, xoff, xD, xfs, xatt, xacc, xsat, xtab, spins, bonds, total;
};
__host__ __device__ inline FusedLayout fused_layout(uint32_t R, uint32_t N, uint32_t dim,
                                                    uint32_t ntab) {
  FusedLayout f;
  f.thr = 0;
  f.wat = f.thr + R * kClasses * 8u;
  f.sof = f.wat + R * 4u;
  f.E = f.sof + R * 4u;
  f.M = f.E + R * 4u;
  f.xoff = f.M + R * 4u;
  f.xD = f.xoff + R * 4u;
  f.xfs = f.xD + R * 4u;
  f.xatt = f.xfs + R * 4u;
  f.xacc = f.xatt + R * 4u;
  f.xsat = (f.xacc + R * 4u + 7u) & ~7u;
  f.xtab = f.xsat + R * 16u;
  f.spins = (f.xtab + ntab * 8u + 15u) & ~15u;
  f.bonds = f.spins + R * N / 2u;                  // four bits per site
  f.total = f.bonds + (dim == 3 ? 3u * N / 2u : 0u);
  return f;
}

// The LDS tables of the single-workgroup kernels (fused and wave plans).
struct FusedTables {
  uint64_t *thr;
  uint32_t *wat, *sof, *xoff, *xD, *xatt, *xacc;
  int32_t *E, *M, *xfs;
  uint64_t *xsat, *xtab;
};

__device__ __forceinline__ FusedTables fused_tables(uint8_t *smem, const FusedLayout &F) {
  FusedTables t;
  t.thr = reinterpret_cast<uint64_t *>(smem + F.thr);
  t.wat = reinterpret_cast<uint32_t *>(smem + F.wat);
  t.sof = reinterpret_cast<uint32_t *>(smem + F.sof);
  t.E = reinterpret_cast<int32_t *>(smem + F.E);
  t.M = reinterpret_cast<int32_t *>(smem + F.M);
  t.xoff = reinterpret_cast<uint32_t *>(smem + F.xoff);
  t.xD = reinterpret_cast<uint32_t *>(smem + F.xD);
  t.xfs = reinterpret_cast<int32_t *>(smem + F.xfs);
  t.xatt = reinterpret_cast<uint32_t *>(smem + F.xatt);
  t.xacc = reinterpret_cast<uint32_t *>(smem + F.xacc);
  t.xsat = reinterpret_cast<uint64_t *>(smem + F.xsat);
  t.xtab = reinterpret_cast<uint64_t *>(smem + F.xtab);
  return t;
}

// Stage every slot's thresholds, the walker/slot maps, E and M, the swap test's
// per-pair data and (ntab > 0) the swap-table rows; the exchange counters start
// at zero and are added to device memory at the end of the launch.
__device__ __forceinline__ void fused_stage(const FusedArgs &a, const FusedTables &t, uint32_t tid,
                                            uint32_t nt) {
  const uint32_t R = a.geo.R;
  for (uint32_t q = tid; q < R * kClasses; q += nt) t.thr[q] = a.st.flip_cmp[q];
  for (uint32_t q = tid; q < R; q += nt) {
    t.wat[q] = a.st.walker_at[q];
    t.sof[q] = a.st.slot_of[q];
    t.E[q] = a.st.E[q];
    t.M[q] = a.st.M[q];
    t.xoff[q] = a.st.swap_off[q];
    t.xD[q] = a.st.swap_D[q];
    t.xfs[q] = a.st.field_sign[q];
    t.xatt[q] = 0u;
    t.xacc[q] = 0u;
    t.xsat[2u * q] = a.st.swap_sat[2u * q];
    t.xsat[2u * q + 1u] = a.st.swap_sat[2u * q + 1u];
  }
  for (uint32_t q = tid; q < a.ntab; q += nt) t.xtab[q] = a.st.swap_tab[q];
}

__device__ __forceinline__ SwapView fused_swap_view(const FusedArgs &a, const FusedTables &t) {
  return SwapView{a.ntab ? t.xtab : a.st.swap_tab, t.xoff, t.xD, t.xsat, a.st.swap_n};
}

// Exchange step e (pairs of parity e & 1) on the LDS maps, pairs spread over
// the threads; E and M of every walker must be in LDS.
__device__ __forceinline__ void fused_exchange(const FusedArgs &a, const FusedTables &t,
                                               const SwapView &sv, uint32_t e, uint32_t tid,
                                               uint32_t nt) {
  const uint32_t R = a.geo.R;
  for (uint32_t kk = (e & 1u) + 2u * tid; kk + 1u < R; kk += 2u * nt) {
    const uint32_t wa = t.wat[kk], wb = t.wat[kk + 1u];
    const uint32_t r = philox(kk, e, 0u, kPurposeSwap, a.key.k0, a.key.k1).x;
    ++t.xatt[kk];
    if ((uint64_t)r < swap_T(sv, kk, t.E[wa] - t.E[wb]) &&
        field_factor(a.st, t.xfs[kk], kk, e, t.M[wa] - t.M[wb], a.key.k0, a.key.k1)) {
      t.wat[kk] = wb;
      t.wat[kk + 1u] = wa;
      t.sof[wa] = kk + 1u;
      t.sof[wb] = kk;
      ++t.xacc[kk];
    }
  }
}

// Maps, E, M and the launch's exchange counts back to device memory.
__device__ __forceinline__ void fused_write_back(const FusedArgs &a, const FusedTables &t,
                                                 uint32_t tid, uint32_t nt) {
  for (uint32_t q = tid; q < a.geo.R; q += nt) {
    a.st.walker_at[q] = t.wat[q];
    a.st.slot_of[q] = t.sof[q];
    a.st.E[q] = t.E[q];
    a.st.M[q] = t.M[q];
    a.st.att[q] += t.xatt[q];
    a.st.acc[q] += t.xacc[q];
  }
}

// PF: every thread holds at most one item (items <= threads), which then stays
// the same for the whole launch.  The draws of sweep s + 1 are computed during
// sweep s with the walker's current slot, off the latency chain of the sweep,
// and recomputed after an exchange step only for walkers whose slot changed.
template <int DIM, int V, bool PF>
__global__ __launch_bounds__(kMaxThreads) void k_fused(FusedArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const Geometry &G = a.geo;
  const uint32_t R = G.R, N = G.N, L = G.L, lgL = a.lg_L;
  const uint32_t lgG = lgL - 3u, gmask = (1u << lgG) - 1u;   // dwords per row
  const uint32_t lgPl = lgL + lgG;                           // dwords per plane (3D)
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const FusedLayout F = fused_layout(R, N, DIM, a.ntab);
  const FusedTables T = fused_tables(smem, F);
  uint64_t *thr = T.thr;
  uint32_t *sof = T.sof;
  int32_t *E = T.E, *M = T.M;
  uint32_t *sp = reinterpret_cast<uint32_t *>(smem + F.spins);   // [R][N/8] nibble dwords
  uint32_t *bx = reinterpret_cast<uint32_t *>(smem + F.bonds), *by = bx + (N >> 3), *bz = by + (N >> 3);

  fused_stage(a, T, tid, nt);
  const SwapView sv = fused_swap_view(a, T);
  unpack_tile_n(sp, a.spins, 0u, (R * N) >> 5, 0xFFFFFFFFu, tid, nt);
  if (DIM == 3) unpack_tile_n(bx, a.st.bonds, 0u, (3u * N) >> 5, 0xFFFFFFFFu, tid, nt);
  __syncthreads();

  const uint32_t smask = (1u << a.lg_spr) - 1u, rmask = G.rows - 1u, imask = (1u << a.lg_items) - 1u;
  const uint32_t shp = a.lg_spr + a.lg_rows;
  const uint32_t items = R << a.lg_items;
  uint32_t rec = a.sch.rec_base, e = a.sch.ex_step;
  // the one item of this thread (PF)
  const bool live = tid < items;
  const uint32_t w1 = live ? tid >> a.lg_items : 0u, li1 = tid & imask;
  const uint32_t g01 = (li1 & smask) * V, y1 = (li1 >> a.lg_spr) & rmask, pl1 = li1 >> shp;
  const uint32_t ctr1 = (((pl1 << a.lg_rows) + y1) << lgG) + g01;
  uint32_t dslot = PF ? sof[w1] : 0u; // slot the draws in rc were taken for
  Words rc[2][V];
  if constexpr (PF) {
#pragma unroll
    for (uint32_t c = 0; c < 2u; ++c)
#pragma unroll
      for (int v = 0; v < V; ++v)
        rc[c][v] = philox(ctr1 + v, a.sch.s0, dslot, c | kPurposeFlip, a.key.k0, a.key.k1);
  }
  for (uint32_t j = 0; j < a.sch.nsw; ++j) {
    const uint32_t s = a.sch.s0 + j;
    const bool do_ex = a.sch.exchange_every && (s + 1u) % a.sch.exchange_every == 0u;
    if constexpr (PF) {
      Words rn[2][V];
      TallyN t = {0u, 0u, 0u};
      const uint32_t pu = (pl1 + L - 1u) & (L - 1u), pd = (pl1 + 1u) & (L - 1u);
      uint32_t *wsp = sp + (size_t)w1 * (N >> 3);
#pragma unroll
      for (uint32_t c = 0; c < 2u; ++c) {
        // the next sweep's draws of this colour, independent of this sweep's work
#pragma unroll
        for (int v = 0; v < V; ++v)
          rn[c][v] = philox(ctr1 + v, s + 1u, dslot, c | kPurposeFlip, a.key.k0, a.key.k1);
        if (live) {
          const uint32_t off = (c + pl1 + (DIM == 3 ? y1 : 0u)) & 1u;
          if constexpr (DIM == 2)
            span2d_n<V>(wsp + (pl1 << lgG), wsp + (pu << lgG), wsp + (pd << lgG), g01, gmask, off,
                        rc[c], thr + dslot * kClasses, t);
          else
            span3d_n<V>(wsp, bx, by, bz, lgG, lgPl, pl1, pu, pd, y1, (y1 + L - 1u) & (L - 1u),
                        (y1 + 1u) & (L - 1u), g01, gmask, off, rc[c], thr + dslot * kClasses, t);
        }
        if (c == 1u && live) { // tallies of both colours, once per sweep
          atomicAdd(&E[w1], a.z2 * (int)t.n - 4 * ((int)t.sc - 8 * (int)t.sb));
          atomicAdd(&M[w1], 4 * (int)t.sb - 2 * (int)t.n);
        }
        __syncthreads();
      }
#pragma unroll
      for (uint32_t c = 0; c < 2u; ++c)
#pragma unroll
        for (int v = 0; v < V; ++v) rc[c][v] = rn[c][v];
    } else {
      for (uint32_t c = 0; c < 2u; ++c) {
        uint32_t cur = 0xFFFFFFFFu;
        TallyN t = {0u, 0u, 0u};
        auto flush = [&]() {
          atomicAdd(&E[cur], a.z2 * (int)t.n - 4 * ((int)t.sc - 8 * (int)t.sb));
          atomicAdd(&M[cur], 4 * (int)t.sb - 2 * (int)t.n);
        };
        for (uint32_t q = tid; q < items; q += nt) {
          const uint32_t w = q >> a.lg_items;
          const uint32_t li = q & imask;
          if (w != cur) {
            if (cur != 0xFFFFFFFFu) flush();
            cur = w;
            t = {0u, 0u, 0u};
          }
          const uint32_t g0 = (li & smask) * V;
          const uint32_t y = (li >> a.lg_spr) & rmask;
          const uint32_t pl = li >> shp;
          const uint32_t pu = (pl + L - 1u) & (L - 1u);
          const uint32_t pd = (pl + 1u) & (L - 1u);
          const uint32_t off = (c + pl + (DIM == 3 ? y : 0u)) & 1u;
          const uint32_t slot = sof[w];
          const uint32_t ctr0 = (((pl << a.lg_rows) + y) << lgG) + g0;
          Words r[V];
#pragma unroll
          for (int v = 0; v < V; ++v)
            r[v] = philox(ctr0 + v, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
          uint32_t *wsp = sp + (size_t)w * (N >> 3);
          if constexpr (DIM == 2)
            span2d_n<V>(wsp + (pl << lgG), wsp + (pu << lgG), wsp + (pd << lgG), g0, gmask, off, r,
                        thr + slot * kClasses, t);
          else
            span3d_n<V>(wsp, bx, by, bz, lgG, lgPl, pl, pu, pd, y, (y + L - 1u) & (L - 1u),
                        (y + 1u) & (L - 1u), g0, gmask, off, r, thr + slot * kClasses, t);
        }
        if (cur != 0xFFFFFFFFu) flush();
        __syncthreads();
      }
    }
    // E and M are final for sweep s (the colour-1 barrier has passed): each
    // walker's thread records them at its slot; only an exchange step needs
    // another barrier (the next sweep's passes touch neither E, M nor the maps)
    if (a.sch.record_every && (s + 1u) % a.sch.record_every == 0u) {
      for (uint32_t v = tid; v < R; v += nt) {
        const uint32_t k = sof[v];
        a.st.E_series[(size_t)rec * R + k] = E[v];
        a.st.M_series[(size_t)rec * R + k] = M[v];
      }
      ++rec;
      // without PF the next colour-0 pass already adds to E and M
      if constexpr (!PF) __syncthreads();
    }
    if (do_ex) {
      __syncthreads(); // records read the maps before the exchange rewrites them
      fused_exchange(a, T, sv, e, tid, nt);
      ++e;
      __syncthreads();
      if constexpr (PF) {
        const uint32_t ns = sof[w1];
        if (ns != dslot) { // the walker moved: its next draws belong to the new slot
          dslot = ns;
#pragma unroll
          for (uint32_t c = 0; c < 2u; ++c)
#pragma unroll
            for (int v = 0; v < V; ++v)
              rc[c][v] = philox(ctr1 + v, s + 1u, dslot, c | kPurposeFlip, a.key.k0, a.key.k1);
        }
      }
    }
  }

  __syncthreads(); // the last exchange's counters
  pack_tile_n(a.spins, sp, (R * N) >> 5, tid, nt);
  fused_write_back(a, T, tid, nt);
}


// Wave plan (2D, L = 8 or 16): walker w's lattice lives in the registers of
// lanes [w G, (w + 1) G) of the workgroup, G = L^2/8, one nibble dword (one
// Philox group) per lane.  G divides 64, so a walker's lanes sit in one
// wavefront and a half sweep takes the rows above and below and the edge dword
// from them with cross-lane moves: no barrier and no LDS traffic for the
// lattice.  At L = 16 lane w G + 16 g + y holds dword g of row y, so the rows
// above and below are the neighbours in the lane's 16-lane DPP row (rotations,
// periodic like the lattice; the stencil adds both, so the direction of a
// rotation does not matter) and the edge dword is lane ^ 16; at L = 8 lane
// w G + y holds row y and the moves are lane permutes.  Each walker's E and M
// stay in its lanes' registers (the changes of a sweep summed over the group);
// thresholds, maps and swap data sit in LDS as in the fused plan, and an
// exchange step takes two barriers.  As in the fused plan the next sweep's
// draws are computed during the current one, off the sweep's dependency chain.
template <int LL>
__global__ __launch_bounds__(kMaxThreads) void k_wave(FusedArgs a) {
  constexpr uint32_t LG_GPR = LL == 16 ? 1u : 0u; // log2 of the dwords per row
  constexpr uint32_t G = LL * LL / 8, NW = LL * LL / 32;        // lanes, packed words per walker
  static_assert(LL == 8 || LL == 16, "wave plan: L = 8 or 16");
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t R = a.geo.R, tid = threadIdx.x, nt = blockDim.x;
  const FusedTables T = fused_tables(smem, fused_layout(R, 0u, 2u, a.ntab));
  fused_stage(a, T, tid, nt);
  const SwapView sv = fused_swap_view(a, T);

  const uint32_t w = tid / G, lw = tid % G; // lane within the walker's group
  const bool live = w < R;
  const uint32_t y = LL == 16 ? (lw & 15u) : lw, g = LL == 16 ? (lw >> 4) : 0u;
  const uint32_t li = (y << LG_GPR) | g; // the group's index: its Philox counter and packed byte
  const uint32_t base = (tid & 63u) & ~(G - 1u); // the walker's first lane in the wavefront (L = 8)
  const int src_up = (int)(base + ((y + LL - 1u) % LL)), src_dn = (int)(base + ((y + 1u) % LL));
  // byte li of the packed lattice holds this dword's 8 sites
  uint8_t *bytes = reinterpret_cast<uint8_t *>(a.spins + (size_t)(live ? w : 0u) * NW);
  uint32_t sw = live ? spread8(bytes[li]) : 0u;
  __syncthreads();

  uint32_t dslot = live ? T.sof[w] : 0u; // the walker's slot (and that of the draws in rc)
  int32_t Ew = live ? T.E[w] : 0, Mw = live ? T.M[w] : 0;
  Words rc[2];
#pragma unroll
  for (uint32_t c = 0; c < 2u; ++c)
    rc[c] = philox(li, a.sch.s0, dslot, c | kPurposeFlip, a.key.k0, a.key.k1);
  uint32_t rec = a.sch.rec_base, e = a.sch.ex_step;
  for (uint32_t j = 0; j < a.sch.nsw; ++j) {
    const uint32_t s = a.sch.s0 + j;
    const uint8_t *tb = reinterpret_cast<const uint8_t *>(T.thr + dslot * kClasses);
    TallyN t = {0u, 0u, 0u};
    Words rn[2];
#pragma unroll
    for (uint32_t c = 0; c < 2u; ++c) {
      rn[c] = philox(li, s + 1u, dslot, c | kPurposeFlip, a.key.k0, a.key.k1);
      const uint32_t off = (c + y) & 1u;
      uint32_t up, dn, ed; // rows y -+ 1, and the row's other dword (the edge the colour sites need)
      if constexpr (LL == 16) {
        up = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)sw, 0x121, 0xF, 0xF, false); // row_ror:1
        dn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)sw, 0x12F, 0xF, 0xF, false); // row_ror:15
        ed = (uint32_t)swap16((int)sw);
      } else {
        up = (uint32_t)__shfl((int)sw, src_up, 64);
        dn = (uint32_t)__shfl((int)sw, src_dn, 64);
        ed = sw; // one dword per row: its own edge, periodic
      }
      const uint32_t l = __builtin_amdgcn_alignbit(sw, ed, 28u);
      const uint32_t rr = __builtin_amdgcn_alignbit(ed, sw, 4u);
      uint32_t u = rr ^ sw;
      u = xad(l, sw, u);
      u = xad(dn, sw, u);
      u = xad(up, sw, u);
      sw = decide_n<true>(sw, u, off, rc[c], tb, t);
    }
    rc[0] = rn[0];
    rc[1] = rn[1];
    // the walker's changes of this sweep, dE in the high half and dM (|dM| <= N
    // < 2^15) in the low half of one sum over its G lanes
    int32_t d = (a.z2 * (int)t.n - 4 * ((int)t.sc - 8 * (int)t.sb)) * 65536 +
                (4 * (int)t.sb - 2 * (int)t.n);
    if constexpr (LL == 16) {
      d = row_sum16(d);
      d += swap16(d);
    } else {
#pragma unroll
      for (uint32_t m = G / 2u; m >= 1u; m >>= 1) d += __shfl_xor(d, (int)m, 64);
    }
    const int32_t dM = ((d & 0xFFFF) ^ 0x8000) - 0x8000;
    Ew += (d - dM) / 65536;
    Mw += dM;
    if (a.sch.record_every && (s + 1u) % a.sch.record_every == 0u) {
      if (live && lw == 0u) {
        a.st.E_series[(size_t)rec * R + dslot] = Ew;
        a.st.M_series[(size_t)rec * R + dslot] = Mw;
      }
      ++rec;
    }
    if (a.sch.exchange_every && (s + 1u) % a.sch.exchange_every == 0u) {
      if (live && lw == 0u) {
        T.E[w] = Ew;
        T.M[w] = Mw;
      }
      __syncthreads();
      fused_exchange(a, T, sv, e, tid, nt);
      ++e;
      __syncthreads();
      const uint32_t ns = live ? T.sof[w] : 0u;
      if (ns != dslot) { // the walker moved: its next draws belong to the new slot
        dslot = ns;
#pragma unroll
        for (uint32_t c = 0; c < 2u; ++c)
          rc[c] = philox(li, s + 1u, dslot, c | kPurposeFlip, a.key.k0, a.key.k1);
      }
    }
  }
  if (live) {
    bytes[li] = (uint8_t)gather8(sw);
    if (lw == 0u) {
      T.E[w] = Ew;
      T.M[w] = Mw;
    }
  }
  __syncthreads();
  fused_write_back(a, T, tid, nt);
}

struct PersistArgs {
  DevState st;
  Geometry geo;
  Keys key;
  Schedule sch;
  uint32_t *spins; // bit-packed, updated in place
  uint32_t lg_L, lg_spr, lg_rows, lg_items;
  uint32_t lg_ipp;     // split plan: log2 of the items of one plane (3D z-plane, 2D row)
  int32_t z2;
  uint32_t spin_limit; // polls of a partner's mailbox before the launch gives up
};

// Persistent replica workgroups: walker w = blockIdx.x keeps its lattice in
// LDS for the whole launch.  After each sweep it folds its own E and M, writes
// its slot's record, and at an exchange step posts (step, E) and (step, M) in
// the mailbox of its slot, waits for the partner slot's posts, and takes the
// same decision as the partner (same draws, same table entries, the field
// factor from the same dM) -- there is no global barrier.
// A partner is at most a few steps apart, so four mailbox generations suffice.
template <int DIM, int V>
__global__ __launch_bounds__(kMaxThreads) void k_persist(PersistArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint64_t s_thr[kClasses];
  __shared__ int s_red[kMaxThreads / 64][2];
  __shared__ uint32_t s_slot, s_stop;
  const Geometry &G = a.geo;
  const uint32_t R = G.R, N = G.N, L = G.L, lgL = a.lg_L;
  const uint32_t lgG = lgL - 3u, gmask = (1u << lgG) - 1u;   // dwords per row
  const uint32_t lgPl = (DIM == 3 ? lgL : 0u) + lgG;          // dwords per plane (3D)
  const uint32_t tid = threadIdx.x, nt = blockDim.x, w = blockIdx.x;
  // four bits per site: spins, then (3D) the x, y, z bond planes, N/8 dwords each
  uint32_t *sp = reinterpret_cast<uint32_t *>(smem);
  uint32_t *bx = sp + (N >> 3), *by = bx + (N >> 3), *bz = by + (N >> 3);
  // every slot's thresholds stay in LDS, so a slot change never waits on memory;
  // the current slot's row is copied to a fixed LDS address for the lookups
  uint64_t *thr = reinterpret_cast<uint64_t *>(sp + (N >> 3) * (DIM == 3 ? 4u : 1u));
  for (uint32_t q = tid; q < R * kClasses; q += nt) thr[q] = a.st.flip_cmp[q];

  uint32_t slot = a.st.slot_of[w];
  int32_t E = a.st.E[w], M = a.st.M[w];
  if (tid < kClasses) s_thr[tid] = a.st.flip_cmp[slot * kClasses + tid];
  unpack_tile_n(sp, a.spins + (size_t)w * (N >> 5), 0u, N >> 5, 0xFFFFFFFFu, tid, nt);
  if (DIM == 3) unpack_tile_n(bx, a.st.bonds, 0u, (3u * N) >> 5, 0xFFFFFFFFu, tid, nt);
  __syncthreads();

  const uint32_t smask = (1u << a.lg_spr) - 1u, rmask = G.rows - 1u;
  const uint32_t shp = a.lg_spr + a.lg_rows;
  const uint32_t items = 1u << a.lg_items;
  uint32_t rec = a.sch.rec_base, e = a.sch.ex_step;
  for (uint32_t j = 0; j < a.sch.nsw; ++j) {
    const uint32_t s = a.sch.s0 + j;
    TallyN t = {0u, 0u, 0u};
    for (uint32_t c = 0; c < 2u; ++c) {
      for (uint32_t q = tid; q < items; q += nt) {
        const uint32_t g0 = (q & smask) * V;
        const uint32_t y = (q >> a.lg_spr) & rmask;
        const uint32_t pl = q >> shp;
        const uint32_t pu = (pl + L - 1u) & (L - 1u);
        const uint32_t pd = (pl + 1u) & (L - 1u);
        const uint32_t off = (c + pl + (DIM == 3 ? y : 0u)) & 1u;
        const uint32_t ctr0 = (((pl << a.lg_rows) + y) << lgG) + g0;
        Words r[V];
#pragma unroll
        for (int v = 0; v < V; ++v)
          r[v] = philox(ctr0 + v, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
        if constexpr (DIM == 2)
          span2d_n<V>(sp + (pl << lgG), sp + (pu << lgG), sp + (pd << lgG), g0, gmask, off, r,
                      s_thr, t);
        else
          span3d_n<V>(sp, bx, by, bz, lgG, lgPl, pl, pu, pd, y, (y + L - 1u) & (L - 1u),
                      (y + 1u) & (L - 1u), g0, gmask, off, r, s_thr, t);
      }
      if (c == 1u) {
        // this wave's energy and magnetisation changes over the sweep, ready
        // at the barrier that ends the sweep
        int dE = a.z2 * (int)t.n - 4 * ((int)t.sc - 8 * (int)t.sb), dM = 4 * (int)t.sb - 2 * (int)t.n;
        dE = wave_total(dE);
        dM = wave_total(dM);
        if ((tid & 63u) == 0u) {
          s_red[tid >> 6][0] = dE;
          s_red[tid >> 6][1] = dM;
        }
      }
      __syncthreads();
    }
    for (uint32_t v = 0; v < (nt >> 6); ++v) {
      E += s_red[v][0];
      M += s_red[v][1];
    }
    const bool do_rec = a.sch.record_every && (s + 1u) % a.sch.record_every == 0u;
    const bool do_ex = a.sch.exchange_every && (s + 1u) % a.sch.exchange_every == 0u;
    if (tid == 0u) {
      // post this slot's energy first, so the partner's wait does not include
      // the record stores below.  The 64-bit word carries the tag and the
      // energy together and the partner reads nothing else of ours, so relaxed
      // agent-scope atomics suffice: no L2 write-back on the post and no L2
      // invalidate per poll.
      uint64_t *mb = a.st.mailbox + (size_t)(e & 3u) * 2u * R; // [slot][E, M]
      const uint64_t tag = (uint64_t)(e + 1u) << 32;
      if (do_ex) {
        __hip_atomic_store(&mb[2u * slot], tag | (uint32_t)E, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if constexpr (DIM == 2) // M for the field factor (2D only)
          __hip_atomic_store(&mb[2u * slot + 1u], tag | (uint32_t)M, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
      if (do_rec) {
        a.st.E_series[(size_t)rec * R + slot] = E;
        a.st.M_series[(size_t)rec * R + slot] = M;
      }
      if (do_ex) {
        uint32_t stop = 0u, nslot = slot;
        const uint32_t par = e & 1u;
        uint32_t partner = 0xFFFFFFFFu;
        if ((slot & 1u) == par && slot + 1u < R) partner = slot + 1u;
        else if ((slot & 1u) != par && slot >= 1u) partner = slot - 1u;
        if (partner != 0xFFFFFFFFu) {
          // everything that does not need the partner's energy before waiting:
          // the pair's draw and its table row
          const uint32_t lo = min(slot, partner);
          const uint32_t r = philox(lo, e, 0u, kPurposeSwap, a.key.k0, a.key.k1).x;
          const PairRow row = pair_row(a.st, lo);
          const int32_t sg = DIM == 2 ? a.st.field_sign[lo] : 0;
          uint64_t v = 0, vm = 0;
          for (uint32_t n = 0;; ++n) {
            // all loads in flight together: one memory round trip per poll
            v = __hip_atomic_load(&mb[2u * partner], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if constexpr (DIM == 2)
              vm = __hip_atomic_load(&mb[2u * partner + 1u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
              vm = tag;
            const uint32_t ab =
                __hip_atomic_load(&a.st.counter[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // the bound and the abort flag first: a limit of 0 gives up at once
            if (n >= a.spin_limit || ab) {
              __hip_atomic_store(&a.st.counter[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              stop = 1u;
              break;
            }
            if ((v & 0xFFFFFFFF00000000ull) == tag && (vm & 0xFFFFFFFF00000000ull) == tag) break;
            __builtin_amdgcn_s_sleep(1);
          }
          if (!stop) {
            const int32_t Ep = (int32_t)(uint32_t)v, Mp = (int32_t)(uint32_t)vm;
            const int32_t Elo = (slot == lo) ? E : Ep, Ehi = (slot == lo) ? Ep : E;
            const int32_t Mlo = (slot == lo) ? M : Mp, Mhi = (slot == lo) ? Mp : M;
            bool accept = (uint64_t)r < pair_T(row, a.st.swap_tab, a.st.swap_n, Elo - Ehi);
            if constexpr (DIM == 2)
              accept = accept && field_factor(a.st, sg, lo, e, Mlo - Mhi, a.key.k0, a.key.k1);
            if (slot == lo) {
              atomicAdd(&a.st.att[lo], 1u);
              if (accept) atomicAdd(&a.st.acc[lo], 1u);
            }
            if (accept) {
              nslot = partner;
              // every lane is waiting at the barrier below: the lookup row
              // can be replaced here, no second barrier needed
              for (uint32_t q = 0; q < kClasses; ++q) s_thr[q] = thr[nslot * kClasses + q];
            }
          }
        }
        s_slot = nslot;
        s_stop = stop;
      }
    }
    if (do_rec) ++rec;
    if (do_ex) {
      ++e;
      __syncthreads();
      if (s_stop) break;
      slot = s_slot;
    }
  }
  pack_tile_n(a.spins + (size_t)w * (N >> 5), sp, N >> 5, tid, nt);
  if (tid == 0u) {
    a.st.E[w] = E;
    a.st.M[w] = M;
    a.st.slot_of[w] = slot;
    a.st.walker_at[slot] = w;
  }
}

// Split persistent walkers: walker w runs as P = NPARTS co-resident
// workgroups, part p owning the Lp = L/P planes [p Lp, (p+1) Lp) -- z-planes in
// 3D, rows in 2D (a "plane" below is either) -- so R walkers fill P R compute
// units.  A part stages two halo planes on each side (local planes 0, 1 and
// Lp+2, Lp+3; its own planes are 2 .. Lp+1).  In the colour-0 half sweep it
// also updates the inner halo plane on each side, with the draws and the
// threshold row the plane's owner uses, so it computes exactly the owner's
// values; colour 1 of its own planes then sees correct neighbours, and one
// exchange of boundary planes per sweep suffices.  At the end of every sweep a
// part posts its two lowest and two highest own planes (bit-packed) and its
// shares of E_int and M, and at an exchange step its E_int share in the slot's
// mailbox beside its M share; each 64-bit word carries its tag (sweep or step + 1) beside 32 bits
// of data, so the reader takes data and tag in one relaxed load and needs no
// fence.  A part reads the lower planes of the part above, the upper planes of
// the part below and the shares of every other part; the parts of both
// walkers of a pair sum the same shares and take the same decision from the
// same draw.  Two generations of posts suffice: a part cannot post sweep s + 2
// before every part has posted s + 1, which each does only after reading every
// post of sweep s.
template <int DIM, int V, int NPARTS>
__global__ __launch_bounds__(kMaxThreads) void k_persist_split(PersistArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint64_t s_thr[kClasses];
  __shared__ int s_red[kMaxThreads / 64][2];
  __shared__ uint32_t s_slot, s_stop, s_ready;
  const Geometry &G = a.geo;
  const uint32_t R = G.R, L = G.L, lgL = a.lg_L, lmask = L - 1u;
  const uint32_t lgG = lgL - 3u, gmask = (1u << lgG) - 1u;  // nibble dwords per row
  const uint32_t lgPl = DIM == 3 ? lgL + lgG : lgG;          // nibble dwords per plane
  constexpr uint32_t P = NPARTS, LGP = NPARTS == 8 ? 3u : NPARTS == 4 ? 2u : 1u;
  static_assert(NPARTS == 2 || NPARTS == 4 || NPARTS == 8, "split plan: 2, 4 or 8 parts");
  const uint32_t Lp = L >> LGP, NP = Lp + 4u;                 // own planes, staged planes
  const uint32_t wpp = G.plane >> 5, nwr = G.N >> 5;         // packed words per plane, per walker
  const uint32_t nb = 4u * wpp, npost = nb + 2u;             // boundary words, words per post
  const uint32_t nread = nb + 2u * (P - 1u);                 // words a part reads per sweep
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t w = blockIdx.x >> LGP, p = blockIdx.x & (P - 1u), z0 = p * Lp;
  const uint32_t pup = (p + 1u) & (P - 1u), pdn = (p + P - 1u) & (P - 1u);
  const uint32_t pdw = NP << lgPl;
  uint32_t *sp = reinterpret_cast<uint32_t *>(smem);
  uint32_t *bx = sp + pdw, *by = bx + pdw, *bz = by + pdw;  // 3D only
  // every slot's table; 3D: 8-byte compare entries, 2D: 4-byte thresholds
  // (the two forms of the decision, see decide_n)
  constexpr bool WIDE = DIM == 3;
  uint32_t *thr = DIM == 3 ? bz + pdw : bx;
  uint32_t *s_tab = reinterpret_cast<uint32_t *>(s_thr); // the current slot's entries
  constexpr uint32_t EW = WIDE ? 2u : 1u;                // dwords per entry
  const uint32_t *src_tab = WIDE ? reinterpret_cast<const uint32_t *>(a.st.flip_cmp) : a.st.flip_thr;
  for (uint32_t q = tid; q < R * kClasses * EW; q += nt) thr[q] = src_tab[q];

  uint32_t slot = a.st.slot_of[w];
  // this part's shares of the walker's E_int and M: part 0 starts from the
  // totals, each part adds the changes of its own sites
  int32_t Es = p ? 0 : a.st.E[w], Ms = p ? 0 : a.st.M[w];
  int32_t Et = a.st.E[w], Mt = a.st.M[w]; // walker totals after the last sweep
  if (tid < kClasses * EW) s_tab[tid] = src_tab[slot * kClasses * EW + tid];
  {
    // planes z0 - 2 .. z0 + Lp + 1, periodic
    const uint32_t f = ((z0 + L - 2u) & lmask) * wpp, cnt = NP * wpp, m = nwr - 1u;
    unpack_tile_n(sp, a.spins + (size_t)w * nwr, f, cnt, m, tid, nt);
    if constexpr (DIM == 3) {
      unpack_tile_n(bx, a.st.bonds, f, cnt, m, tid, nt);
      unpack_tile_n(by, a.st.bonds + nwr, f, cnt, m, tid, nt);
      unpack_tile_n(bz, a.st.bonds + 2u * nwr, f, cnt, m, tid, nt);
    }
  }
  __syncthreads();

  const uint32_t smask = (1u << a.lg_spr) - 1u;
  uint32_t rec = a.sch.rec_base, e = a.sch.ex_step;
  // Own-plane item q of colour c in sweep s: V groups of plane 2 + (q >> lg_ipp).
  auto own_item = [&](uint32_t q, uint32_t s, uint32_t c, TallyN &t) {
    const uint32_t lp = 2u + (q >> a.lg_ipp);
    const uint32_t g0 = (q & smask) * V;
    const uint32_t y = DIM == 3 ? (q >> a.lg_spr) & lmask : 0u;
    const uint32_t z = (z0 + lp + L - 2u) & lmask; // global plane
    const uint32_t off = (c + lp + y) & 1u;         // z0 is even
    const uint32_t ctr0 = DIM == 3 ? (((z << lgL) + y) << lgG) + g0 : (z << lgG) + g0;
    Words r[V];
#pragma unroll
    for (int v = 0; v < V; ++v)
      r[v] = philox(ctr0 + v, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
    if constexpr (DIM == 3)
      span3d_n<V, WIDE>(sp, bx, by, bz, lgG, lgPl, lp, lp - 1u, lp + 1u, y, (y + L - 1u) & lmask,
                        (y + 1u) & lmask, g0, gmask, off, r, s_thr, t);
    else
      span2d_n<V, WIDE>(sp + (lp << lgPl), sp + ((lp - 1u) << lgPl), sp + ((lp + 1u) << lgPl), g0,
                        gmask, off, r, s_thr, t);
  };
  // The end of sweep s for wave 0 (tid < 64): post this part's boundary planes
  // and shares, wait for the neighbours' and (exchange step) the partner's,
  // receive the halo planes, record, decide.  Leaves s_slot and s_stop.
  auto handshake = [&](uint32_t s, bool do_rec, bool do_ex, uint32_t rec_i) {
    for (uint32_t v = 0; v < (nt >> 6); ++v) {
      Es += s_red[v][0];
      Ms += s_red[v][1];
    }
    const uint64_t hi = 0xFFFFFFFF00000000ull;
    const uint64_t tag = (uint64_t)(s + 1u) << 32, etag = (uint64_t)(e + 1u) << 32;
    // the posts of this sweep's generation for walker w, one per part
    uint64_t *posts = a.st.halo + ((size_t)(s & 1u) * R + w) * P * npost;
    uint64_t *mine = posts + (size_t)p * npost;
    uint64_t *mb = a.st.mailbox + (size_t)(e & 3u) * 2u * P * R; // [slot][part][E, M]
    // post: words [0, 2 wpp) = own planes 2, 3; [2 wpp, 4 wpp) = planes Lp, Lp + 1
    for (uint32_t q = tid; q < nb; q += 64u) {
      const bool lo = q < 2u * wpp;
      const uint4 x = reinterpret_cast<const uint4 *>(sp + ((lo ? 2u : Lp) << lgPl))[lo ? q : q - 2u * wpp];
      const uint32_t word =
          gather8(x.x) | (gather8(x.y) << 8) | (gather8(x.z) << 16) | (gather8(x.w) << 24);
      __hip_atomic_store(mine + q, tag | word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t partner = 0xFFFFFFFFu;
    if (do_ex) {
      const uint32_t par = e & 1u;
      if ((slot & 1u) == par && slot + 1u < R) partner = slot + 1u;
      else if ((slot & 1u) != par && slot >= 1u) partner = slot - 1u;
    }
    if (tid == 0u) {
      if (do_ex) {
        __hip_atomic_store(&mb[2u * (P * slot + p)], etag | (uint32_t)Es, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        if constexpr (DIM == 2) // M for the field factor (2D only)
          __hip_atomic_store(&mb[2u * (P * slot + p) + 1u], etag | (uint32_t)Ms, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
      __hip_atomic_store(mine + nb, tag | (uint32_t)Es, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(mine + nb + 1u, tag | (uint32_t)Ms, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    // everything of the swap test that does not need the energies, before waiting
    uint32_t lo = 0u, rr = 0u;
    int32_t sg = 0;
    PairRow row{0, 0u, 0u, 0u};
    if (tid == 0u && partner != 0xFFFFFFFFu) {
      lo = min(slot, partner);
      rr = philox(lo, e, 0u, kPurposeSwap, a.key.k0, a.key.k1).x;
      row = pair_row(a.st, lo);
      if constexpr (DIM == 2) sg = a.st.field_sign[lo];
    }
    // Word q of what this part reads: the lower boundary planes of the part
    // above (q < 2 wpp, its post words q), the upper ones of the part below
    // (2 wpp <= q < 4 wpp), then the E_int and M shares of the other parts.
    uint32_t src[kSplitWordsPerLane]; // word offsets from posts
    uint32_t pend = 0u;
#pragma unroll
    for (uint32_t k = 0; k < kSplitWordsPerLane; ++k) {
      const uint32_t q = min(tid + 64u * k, nread - 1u);
      if (tid + 64u * k < nread) pend |= 1u << k;
      if (q < 2u * wpp) src[k] = pup * npost + q;
      else if (q < nb) src[k] = pdn * npost + q;
      else {
        const uint32_t i = q - nb;
        src[k] = ((p + 1u + (i >> 1)) & (P - 1u)) * npost + nb + (i & 1u);
      }
    }
    // wait for those and, at an exchange step, the partner slot's E and M shares.
    // Every round issues all of a lane's loads before testing any (one memory
    // round trip per round); a word is consumed when its tag arrives and
    // cannot change again before this part has posted its next sweep, so
    // reloading a consumed word is harmless (loading only the words still
    // pending was measured 0.7% slower: the masked loads cost more than the
    // re-read words, which are a few MB per launch beside 8 TB/s).
    // lane k < 2P reads word k of the partner slot's posts (E and M shares by
    // part); in 3D, without a field, lane k < P reads part k's E share only
    constexpr uint32_t NW = DIM == 2 ? 2u * P : P;
    uint32_t ppend = (partner != 0xFFFFFFFFu && tid < NW) ? 1u : 0u;
    const uint32_t pw = DIM == 2 ? (tid & (2u * P - 1u)) : 2u * (tid & (P - 1u));
    const uint64_t *pmb = &mb[2u * P * (partner != 0xFFFFFFFFu ? partner : slot) + pw];
    int32_t sE = 0, sM = 0, pE = 0;
    uint32_t stop = 0u;
    for (uint32_t n = 0;; ++n) {
      uint64_t v[kSplitWordsPerLane];
#pragma unroll
      for (uint32_t k = 0; k < kSplitWordsPerLane; ++k)
        v[k] = __hip_atomic_load(posts + src[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t pv = __hip_atomic_load(pmb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t ab =
          __hip_atomic_load(&a.st.counter[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (uint32_t k = 0; k < kSplitWordsPerLane; ++k) {
        if (!((pend >> k) & 1u) || (v[k] & hi) != tag) continue;
        pend &= ~(1u << k);
        const uint32_t q = tid + 64u * k, x = (uint32_t)v[k];
        if (q < nb) {
          // the part above's lowest planes are this part's upper halo, the
          // part below's highest planes the lower halo
          const bool lo = q < 2u * wpp;
          reinterpret_cast<uint4 *>(sp + (lo ? ((Lp + 2u) << lgPl) : 0u))[lo ? q : q - 2u * wpp] =
              make_uint4(spread8(x & 0xFFu), spread8(__builtin_amdgcn_ubfe(x, 8u, 8u)),
                         spread8(__builtin_amdgcn_ubfe(x, 16u, 8u)), spread8(x >> 24));
        } else if (((q - nb) & 1u) == 0u) {
          sE += (int32_t)x;
        } else {
          sM += (int32_t)x;
        }
      }
      if (ppend && (pv & hi) == etag) {
        ppend = 0u;
        pE = (int32_t)(uint32_t)pv;
      }
      // the bound and the abort flag first: a limit of 0 gives up at once
      if (n >= a.spin_limit || __any(ab != 0u)) {
        if (tid == 0u)
          __hip_atomic_store(&a.st.counter[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        stop = 1u;
        break;
      }
      if (!__any((pend | ppend) != 0u)) break;
      __builtin_amdgcn_s_sleep(1);
    }
    {
      // the other parts' shares arrived in lanes sl .. sl + 2(P-1) - 1 of
      // one load round (E at even offsets, M at odd; the launch checks that
      // they do not wrap past lane 63): read them directly
      const int sl = (int)(nb & 63u);
      int32_t tE = 0, tM = 0;
#pragma unroll
      for (uint32_t i = 0; i + 1u < P; ++i) {
        tE += __shfl(sE, sl + 2 * (int)i, 64);
        tM += __shfl(sM, sl + 2 * (int)i + 1, 64);
      }
      sE = tE;
      sM = tM;
    }
    // the partner slot's P shares of E (even lanes 0 .. 2P-2) and of M (odd
    // lanes): independent reads
    int32_t Ep = 0, Mp = 0;
#pragma unroll
    for (uint32_t k = 0; k < P; ++k) {
      if constexpr (DIM == 2) {
        Ep += __shfl(pE, (int)(2u * k), 64);
        Mp += __shfl(pE, (int)(2u * k + 1u), 64);
      } else {
        Ep += __shfl(pE, (int)k, 64);
      }
    }
    if (tid == 0u) {
      Et = Es + sE;
      Mt = Ms + sM;
      uint32_t nslot = slot;
      if (!stop) {
        if (do_rec && p == 0u) {
          a.st.E_series[(size_t)rec_i * R + slot] = Et;
          a.st.M_series[(size_t)rec_i * R + slot] = Mt;
        }
        if (partner != 0xFFFFFFFFu) {
          const int32_t Elo = (slot == lo) ? Et : Ep, Ehi = (slot == lo) ? Ep : Et;
          const int32_t Mlo = (slot == lo) ? Mt : Mp, Mhi = (slot == lo) ? Mp : Mt;
          bool accept = (uint64_t)rr < pair_T(row, a.st.swap_tab, a.st.swap_n, Elo - Ehi);
          if constexpr (DIM == 2)
            accept = accept && field_factor(a.st, sg, lo, e, Mlo - Mhi, a.key.k0, a.key.k1);
          if (slot == lo && p == 0u) {
            atomicAdd(&a.st.att[lo], 1u);
            if (accept) atomicAdd(&a.st.acc[lo], 1u);
          }
          if (accept) {
            nslot = partner;
            for (uint32_t q = 0; q < kClasses * EW; ++q) s_tab[q] = thr[nslot * kClasses * EW + q];
          }
        }
      }
      s_slot = nslot;
      s_stop = stop;
    }
  };

  // After a sweep that ends without an exchange step the handshake is not
  // waited for: the next sweep's colour-0 pass starts at once on the planes
  // that neither the post reads nor the halo feeds (4 .. Lp - 1) while wave 0
  // posts and waits, and the other planes follow once wave 0 has received the
  // halo (s_ready).  After an exchange step the next sweep needs the decision
  // (its slot, its draws), so every wave waits for the handshake as before.
  // 2D only: the 3D kernel measured faster without this path compiled in.
  if (tid == 0u) s_ready = 0xFFFFFFFFu;
  __syncthreads();
  bool pending = false;
  uint32_t ps = 0u, prec = 0u;
  bool prec_do = false;
  const uint32_t ipp = 1u << a.lg_ipp;
  for (uint32_t j = 0; j < a.sch.nsw; ++j) {
    const uint32_t s = a.sch.s0 + j;
    TallyN t = {0u, 0u, 0u};
    // colour 0: own planes 2 .. Lp + 1, V groups per item
    if (DIM == 2 && pending) {
      if (tid < 64u) {
        handshake(ps, prec_do, false, prec);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup"); // the halo planes, before the flag
        if (tid == 0u) __hip_atomic_store(&s_ready, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      for (uint32_t q = tid; q < ((Lp - 4u) << a.lg_ipp); q += nt) own_item(q + (2u << a.lg_ipp), s, 0u, t);
      while (__hip_atomic_load(&s_ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != s)
        __builtin_amdgcn_s_sleep(1);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      // own planes 0, 1, Lp - 2, Lp - 1 (local 2, 3, Lp, Lp + 1), from the last
      // thread down: those have the fewest items above
      for (uint32_t q = nt - 1u - tid; q < 4u * ipp; q += nt) {
        const uint32_t k = q >> a.lg_ipp, own = k < 2u ? k : Lp - 4u + k;
        own_item((own << a.lg_ipp) | (q & (ipp - 1u)), s, 0u, t);
      }
    } else {
      for (uint32_t q = tid; q < (Lp << a.lg_ipp); q += nt) own_item(q, s, 0u, t);
    }
    {
      // the inner halo planes (local 1 and Lp + 2), one group per item on
      // the first waves: one such wave per SIMD keeps the pass balanced.
      // Their flips are their owners' to count.
      const uint32_t gpp = 1u << lgPl; // groups per plane
      for (uint32_t q = tid; q < 2u * gpp; q += nt) {
        const uint32_t lp = q < gpp ? 1u : Lp + 2u;
        const uint32_t g0 = q & gmask;
        const uint32_t y = DIM == 3 ? (q >> lgG) & lmask : 0u;
        const uint32_t z = (z0 + lp + L - 2u) & lmask;
        const uint32_t off = (lp + y) & 1u;
        const uint32_t ctr = DIM == 3 ? (((z << lgL) + y) << lgG) + g0 : (z << lgG) + g0;
        Words r[1];
        r[0] = philox(ctr, s, slot, kPurposeFlip, a.key.k0, a.key.k1);
        TallyN tl = {0u, 0u, 0u};
        if constexpr (DIM == 3)
          span3d_n<1, WIDE>(sp, bx, by, bz, lgG, lgPl, lp, lp - 1u, lp + 1u, y, (y + L - 1u) & lmask,
                            (y + 1u) & lmask, g0, gmask, off, r, s_thr, tl);
        else
          span2d_n<1, WIDE>(sp + (lp << lgPl), sp + ((lp - 1u) << lgPl), sp + ((lp + 1u) << lgPl), g0,
                            gmask, off, r, s_thr, tl);
      }
    }
    __syncthreads();
    if (pending) {
      pending = false;
      if (s_stop) break;
    }
    // colour 1
    for (uint32_t q = tid; q < (Lp << a.lg_ipp); q += nt) own_item(q, s, 1u, t);
    {
      // this wave's energy and magnetisation changes over the sweep, ready
      // at the barrier that ends the sweep
      int dE = a.z2 * (int)t.n - 4 * ((int)t.sc - 8 * (int)t.sb), dM = 4 * (int)t.sb - 2 * (int)t.n;
      dE = wave_total(dE);
      dM = wave_total(dM);
      if ((tid & 63u) == 0u) {
        s_red[tid >> 6][0] = dE;
        s_red[tid >> 6][1] = dM;
      }
    }
    __syncthreads();
    const bool do_rec = a.sch.record_every && (s + 1u) % a.sch.record_every == 0u;
    const bool do_ex = a.sch.exchange_every && (s + 1u) % a.sch.exchange_every == 0u;
    if (DIM == 2 && !do_ex && j + 1u < a.sch.nsw) {
      pending = true;
      ps = s;
      prec = rec;
      prec_do = do_rec;
    } else {
      if (tid < 64u) handshake(s, do_rec, do_ex, rec);
      __syncthreads();
      if (s_stop) break;
      slot = s_slot;
    }
    if (do_rec) ++rec;
    if (do_ex) ++e;
  }
  pack_tile_n(a.spins + (size_t)w * nwr + z0 * wpp, sp + (2u << lgPl), Lp * wpp, tid, nt);
  if (tid == 0u && p == 0u) {
    a.st.E[w] = Et;
    a.st.M[w] = Mt;
    a.st.slot_of[w] = slot;
    a.st.walker_at[slot] = w;
  }
}

// ---- one walker per lane (the paper's decomposition) -----------------------
// Lane w holds walker w's bit-packed lattice in registers (N/32 words, bit i =
// site i, as in HBM) and visits its colour-c sites one after another; the
// workgroup's LDS holds every slot's thresholds, the walkers' E and M and the
// walker/slot maps for the exchange steps.  All indexing is unrolled at
// compile time for the lattice side L.
template <int L>
__device__ __forceinline__ uint32_t lane_bit(const uint32_t (&S)[L * L / 32], int x, int y) {
  const int i = ((y + L) % L) * L + ((x + L) % L);
  return (S[i >> 5] >> (i & 31)) & 1u;
}

template <int L>
__global__ __launch_bounds__(kMaxThreads) void k_lanes(FusedArgs a) {
  constexpr int NW = L * L / 32, GPR = L / 8;
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t R = a.geo.R, tid = threadIdx.x, nt = blockDim.x;
  uint32_t *thr = reinterpret_cast<uint32_t *>(smem);        // [R][16]
  int32_t *E = reinterpret_cast<int32_t *>(thr + R * kClasses); // [R] by walker
  int32_t *M = E + R;
  uint32_t *wat = reinterpret_cast<uint32_t *>(M + R);
  uint32_t *sof = wat + R;
  for (uint32_t q = tid; q < R * kClasses; q += nt) thr[q] = a.st.flip_thr[q];
  for (uint32_t q = tid; q < R; q += nt) {
    E[q] = a.st.E[q];
    M[q] = a.st.M[q];
    wat[q] = a.st.walker_at[q];
    sof[q] = a.st.slot_of[q];
  }
  const bool live = tid < R;
  const uint32_t w = tid;
  uint32_t S[NW];
#pragma unroll
  for (int j = 0; j < NW; ++j) S[j] = live ? a.spins[(size_t)w * NW + j] : 0u;
  __syncthreads();
  int32_t e = live ? E[w] : 0, m = live ? M[w] : 0;
  uint32_t rec = a.sch.rec_base, ex = a.sch.ex_step;
  for (uint32_t j = 0; j < a.sch.nsw; ++j) {
    const uint32_t s = a.sch.s0 + j;
    const uint32_t slot = live ? sof[w] : 0u;
    if (live) {
      const uint32_t *T = thr + slot * kClasses;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int y = 0; y < L; ++y) {
          const int off = (c + y) & 1;
#pragma unroll
          for (int g = 0; g < GPR; ++g) {
            const Words r = philox((uint32_t)(y * GPR + g), s, slot, (uint32_t)c | kPurposeFlip,
                                   a.key.k0, a.key.k1);
            const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
            for (int mm = 0; mm < 4; ++mm) {
              const int x = 8 * g + off + 2 * mm, i = y * L + x;
              const uint32_t b = lane_bit<L>(S, x, y);
              const uint32_t nb = lane_bit<L>(S, x - 1, y) + lane_bit<L>(S, x + 1, y) +
                                  lane_bit<L>(S, x, y - 1) + lane_bit<L>(S, x, y + 1);
              const uint32_t u = b ? 4u - nb : nb;        // neighbours unlike the site
              if (rw[mm] <= T[8u * b + u]) {
                S[i >> 5] ^= 1u << (i & 31);
                e += 8 - 4 * (int32_t)u;                  // dE_int = 2z - 4u
                m += 4 * (int32_t)b - 2;                  // dM = -2 s
              }
            }
          }
        }
      }
      if (a.sch.record_every && (s + 1u) % a.sch.record_every == 0u) {
        a.st.E_series[(size_t)rec * R + slot] = e;
        a.st.M_series[(size_t)rec * R + slot] = m;
      }
    }
    if (a.sch.record_every && (s + 1u) % a.sch.record_every == 0u) ++rec;
    if (a.sch.exchange_every && (s + 1u) % a.sch.exchange_every == 0u) {
      if (live) {
        E[w] = e;
        M[w] = m;
      }
      __syncthreads();
      exchange_step(a.st, R, a.key.k0, a.key.k1, ex, E, M, wat, sof, tid, nt);
      ++ex;
      __syncthreads();
    }
  }
#pragma unroll
  for (int j = 0; j < NW; ++j)
    if (live) a.spins[(size_t)w * NW + j] = S[j];
  if (live) {
    a.st.E[w] = e;
    a.st.M[w] = m;
  }
  __syncthreads();
  for (uint32_t q = tid; q < R; q += nt) {
    a.st.walker_at[q] = wat[q];
    a.st.slot_of[q] = sof[q];
  }
}

// ---- batched form ----------------------------------------------------------
// LDS layout of a batched-sweep workgroup holding W walkers of one instance.
struct BatchLayout {
  uint32_t thr, slot, E, M, acc, spins, bonds, total;
};
__host__ __device__ inline BatchLayout batch_layout(uint32_t W, uint32_t N, uint32_t dim) {
  BatchLayout b;
  b.thr = 0;
  b.slot = b.thr + W * kClasses * 8u;
  b.E = b.slot + W * 4u;
  b.M = b.E + W * 4u;
  b.acc = b.M + W * 4u;
  b.spins = (b.acc + W * 8u + 15u) & ~15u;
  b.bonds = b.spins + W * N / 2u;                  // four bits per site
  b.total = b.bonds + (dim == 3 ? 3u * N / 2u : 0u);
  return b;
}


// Batched sweep, one workgroup = walkers [w0, w0 + W) of one instance whole
// in LDS at four bits per site (EA: with the instance's bond planes), the
// cycle's sweeps in place, per-walker E and M, records by slot.
template <int DIM, int V>
__global__ __launch_bounds__(kMaxThreads) void k_batch_sweep(const BatchInst *insts,
                                                             const BatchItem *items, uint32_t W,
                                                             uint32_t K) {
  extern __shared__ __align__(16) uint8_t smem[];
  const BatchItem it = items[blockIdx.x];
  const BatchInst &I = insts[it.inst];
  const uint32_t nsw = cycle_sweeps(I.ctr, K);
  if (nsw == 0u) return;
  const uint32_t s0 = I.ctr[kCtrSweeps];
  const Geometry &G = I.geo;
  const uint32_t R = G.R, N = G.N, L = G.L, lgL = I.lg_L;
  const uint32_t lgG = lgL - 3u, gmask = (1u << lgG) - 1u;   // dwords per row
  const uint32_t lgPl = lgL + lgG;                           // dwords per plane (3D)
  const uint32_t nw = min(W, R - it.w0);
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const BatchLayout B = batch_layout(W, N, DIM);
  uint64_t *thr = reinterpret_cast<uint64_t *>(smem + B.thr);
  uint32_t *slot = reinterpret_cast<uint32_t *>(smem + B.slot);
  int32_t *E = reinterpret_cast<int32_t *>(smem + B.E);
  int32_t *M = reinterpret_cast<int32_t *>(smem + B.M);
  int32_t *acc = reinterpret_cast<int32_t *>(smem + B.acc);
  uint32_t *sp = reinterpret_cast<uint32_t *>(smem + B.spins);
  uint32_t *bx = reinterpret_cast<uint32_t *>(smem + B.bonds), *by = bx + (N >> 3), *bz = by + (N >> 3);

  for (uint32_t v = tid; v < nw; v += nt) {
    slot[v] = I.st.slot_of[it.w0 + v];
    E[v] = I.st.E[it.w0 + v];
    M[v] = I.st.M[it.w0 + v];
    acc[2u * v] = 0;
    acc[2u * v + 1u] = 0;
  }
  __syncthreads();
  for (uint32_t q = tid; q < nw * kClasses; q += nt)
    thr[q] = I.st.flip_cmp[slot[q / kClasses] * kClasses + (q % kClasses)];
  unpack_tile_n(sp, I.st.spins[0] + (size_t)it.w0 * (N >> 5), 0u, (nw * N) >> 5, 0xFFFFFFFFu, tid, nt);
  if (DIM == 3) unpack_tile_n(bx, I.st.bonds, 0u, (3u * N) >> 5, 0xFFFFFFFFu, tid, nt);
  __syncthreads();

  const uint32_t smask = (1u << I.lg_spr) - 1u, rmask = G.rows - 1u, imask = (1u << I.lg_items) - 1u;
  const uint32_t shp = I.lg_spr + I.lg_rows;
  const uint32_t items_n = nw << I.lg_items;
  const uint32_t wdw = N >> 3;                                  // LDS dwords per walker
  uint32_t rec = I.ctr[kCtrRecords];
  for (uint32_t j = 0; j < nsw; ++j) {
    const uint32_t s = s0 + j;
    for (uint32_t c = 0; c < 2u; ++c) {
      uint32_t cur = 0xFFFFFFFFu;
      TallyN t = {0u, 0u, 0u};
      auto flush = [&]() {
        atomicAdd(&acc[2u * cur], I.z2 * (int)t.n - 4 * ((int)t.sc - 8 * (int)t.sb));
        atomicAdd(&acc[2u * cur + 1u], 4 * (int)t.sb - 2 * (int)t.n);
      };
      for (uint32_t q = tid; q < items_n; q += nt) {
        const uint32_t v = q >> I.lg_items;
        const uint32_t li = q & imask;
        if (v != cur) {
          if (cur != 0xFFFFFFFFu) flush();
          cur = v;
          t = {0u, 0u, 0u};
        }
        const uint32_t g0 = (li & smask) * V;
        const uint32_t y = (li >> I.lg_spr) & rmask;
        const uint32_t pl = li >> shp;
        const uint32_t pu = (pl + L - 1u) & (L - 1u);
        const uint32_t pd = (pl + 1u) & (L - 1u);
        const uint32_t off = (c + pl + (DIM == 3 ? y : 0u)) & 1u;
        const uint32_t ctr0 = (((pl << I.lg_rows) + y) << lgG) + g0;
        Words r[V];
#pragma unroll
        for (int u = 0; u < V; ++u)
          r[u] = philox(ctr0 + u, s, slot[v], c | kPurposeFlip, I.key.k0, I.key.k1);
        uint32_t *wsp = sp + (size_t)v * wdw;
        if constexpr (DIM == 2)
          span2d_n<V>(wsp + (pl << lgG), wsp + (pu << lgG), wsp + (pd << lgG), g0, gmask, off, r,
                      thr + v * kClasses, t);
        else
          span3d_n<V>(wsp, bx, by, bz, lgG, lgPl, pl, pu, pd, y, (y + L - 1u) & (L - 1u),
                      (y + 1u) & (L - 1u), g0, gmask, off, r, thr + v * kClasses, t);
      }
      if (cur != 0xFFFFFFFFu) flush();
      __syncthreads();
    }
    for (uint32_t v = tid; v < nw; v += nt) {
      E[v] += acc[2u * v];
      M[v] += acc[2u * v + 1u];
      acc[2u * v] = 0;
      acc[2u * v + 1u] = 0;
      if (I.record_every && (s + 1u) % I.record_every == 0u) {
        I.st.E_series[(size_t)rec * R + slot[v]] = E[v];
        I.st.M_series[(size_t)rec * R + slot[v]] = M[v];
      }
    }
    if (I.record_every && (s + 1u) % I.record_every == 0u) ++rec;
    __syncthreads();
  }
  pack_tile_n(I.st.spins[0] + (size_t)it.w0 * (N >> 5), sp, (nw * N) >> 5, tid, nt);
  for (uint32_t v = tid; v < nw; v += nt) {
    I.st.E[it.w0 + v] = E[v];
    I.st.M[it.w0 + v] = M[v];
  }
}

// One thread per (instance, pair k): the pair's decision when the instance's
// cycle ends on an exchange step and k has the step's parity.
__global__ void k_batch_exchange(const BatchInst *insts, const uint2 *pairs, uint32_t n_pairs,
                                 uint32_t K) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_pairs) return;
  const uint2 p = pairs[q];
  const BatchInst &I = insts[p.x];
  const uint32_t nsw = cycle_sweeps(I.ctr, K);
  const uint32_t every = I.ctr[kCtrEvery], e = I.ctr[kCtrExchanges];
  if (nsw == 0u || every == 0u || (I.ctr[kCtrSweeps] + nsw) % every != 0u) return;
  if ((p.y & 1u) != (e & 1u)) return;
  exchange_pair(I.st, p.y, I.key.k0, I.key.k1, e, I.st.E, I.st.M, I.st.walker_at, I.st.slot_of);
}

__global__ void k_batch_target(const BatchInst *insts, uint32_t n, uint32_t add, uint32_t every) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t *ctr = insts[i].ctr;
  ctr[kCtrTarget] = ctr[kCtrSweeps] + add;
  ctr[kCtrActive] = add ? 1u : 0u;
  ctr[kCtrEvery] = every;
}

// One thread per instance: advance the schedule by this cycle's sweeps (and,
// for a tiled instance, switch to the spin buffer the cycle wrote).
__global__ void k_batch_advance(const BatchInst *insts, const uint32_t *list, uint32_t n,
                                uint32_t K) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const BatchInst &I = insts[list ? list[q] : q];
  uint32_t *ctr = I.ctr;
  const uint32_t nsw = cycle_sweeps(ctr, K);
  if (nsw == 0u) return;
  const uint32_t s0 = ctr[kCtrSweeps], every = ctr[kCtrEvery];
  if (I.record_every) ctr[kCtrRecords] += (s0 + nsw) / I.record_every - s0 / I.record_every;
  if (every && (s0 + nsw) % every == 0u) ctr[kCtrExchanges] += 1u;
  if (ctr[kCtrTiles] > 1u) ctr[kCtrCur] ^= 1u;
  ctr[kCtrSweeps] = s0 + nsw;
  if (s0 + nsw >= ctr[kCtrTarget]) ctr[kCtrActive] = 0u;
}

__global__ void k_exchange(DevState st, uint32_t R, Keys key, uint32_t e) {
  exchange_step(st, R, key.k0, key.k1, e, st.E, st.M, st.walker_at, st.slot_of,
                blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// Initial spins: site i of walker w takes word i mod 4 of block (i/4, w, 0, spin
// purpose); top bit set = down.  upload: convert caller-provided +-1 bytes.
// One thread per 32-site word of the packed lattice.
__global__ void k_init_spins(DevState st, Geometry G, Keys key, uint32_t upload) {
  const uint32_t nwr = G.nwr;
  const uint64_t total = (uint64_t)nwr * G.R;
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < total;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t w = (uint32_t)(q / nwr), i0 = 32u * (uint32_t)(q % nwr);
    const uint32_t n = min(32u, G.N - i0); // sites in this word (the last may be partial)
    uint32_t bits = 0;
    if (upload) {
      const uint8_t *src = st.staging + (size_t)w * G.N + i0;
      for (uint32_t j = 0; j < n; ++j) bits |= (uint32_t)((src[j] >> 7) & 1u) << j;
    } else {
#pragma unroll
      for (uint32_t j = 0; j < 8u; ++j) {
        const Words r = philox((i0 >> 2) + j, w, 0u, kPurposeSpin, key.k0, key.k1);
        bits |= ((r.x >> 31) | ((r.y >> 31) << 1) | ((r.z >> 31) << 2) | ((r.w >> 31) << 3)) << (4u * j);
      }
      if (n < 32u) bits &= (1u << n) - 1u;
    }
    st.spins[0][q] = bits;
  }
}

// EA couplings: bond b = 3 i + d takes word b mod 4 of block (b/4, 0, 0, bond
// purpose); stored as bit-packed planes [3][N], bit set = J -1.
__global__ void k_init_bonds(DevState st, Geometry G, Keys key, uint32_t upload) {
  const uint32_t wpr = G.N >> 5, total = 3u * wpr;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    const uint32_t d = q / wpr, i0 = 32u * (q % wpr);
    uint32_t bits = 0;
    for (uint32_t j = 0; j < 32u; ++j) {
      uint32_t v;
      if (upload) {
        v = (st.staging[(size_t)d * G.N + i0 + j] >> 7) & 1u;
      } else {
        const uint32_t b = 3u * (i0 + j) + d;
        const Words r = philox(b >> 2, 0u, 0u, kPurposeBond, key.b0, key.k1);
        const uint32_t word = (b & 3u) == 0 ? r.x : (b & 3u) == 1 ? r.y : (b & 3u) == 2 ? r.z : r.w;
        v = word >> 31;
      }
      bits |= v << j;
    }
    st.bonds[q] = bits;
  }
}

__global__ void k_reset(DevState st, Geometry G, uint32_t halo_words) {
  const uint32_t R = G.R;
  // posts are matched by their tags: none may survive from an earlier use of the memory
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < halo_words; q += gridDim.x * blockDim.x)
    st.halo[q] = 0;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < kMaxSweepsPerLaunch * R * 4u;
       q += gridDim.x * blockDim.x) {
    st.acc3[q] = 0;
    if (q < R) {
      st.walker_at[q] = q;
      st.slot_of[q] = q;
      st.E[q] = 0;
      st.M[q] = 0;
      st.att[q] = 0;
      st.acc[q] = 0;
    }
    if (q < 4u) st.counter[q] = 0;
  }
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < 8u * kMaxParts * R;
       q += gridDim.x * blockDim.x)
    st.mailbox[q] = 0;
}

__device__ __forceinline__ uint32_t bit_at(const uint32_t *words, uint32_t i) {
  return (words[i >> 5] >> (i & 31u)) & 1u;
}

// Full recount of E_int and M of every walker from spin buffer cur.
// Word-level recount for rows of at least 32 sites: one thread per packed word
// (32 sites of one row); unsatisfied bonds to the +x, +y (, +z) neighbours are
// popcounts of XORs with the shifted neighbour words (and the couplings), and
// E_int = sum over bonds (2 [unsatisfied] - 1), M = 32 - 2 popcount per word.
template <int DIM>
__global__ void k_recount_words(DevState st, Geometry G, uint32_t cur) {
  const uint32_t w = blockIdx.y;
  const uint32_t nwr = G.N >> 5, wpr = G.L >> 5, wpp = (G.L * G.L) >> 5;
  const uint32_t *sp = st.spins[cur] + (size_t)w * nwr;
  int e = 0, m = 0;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nwr; q += gridDim.x * blockDim.x) {
    const uint32_t a = sp[q];
    const uint32_t rs = q - q % wpr;                           // first word of the row
    const uint32_t nx = sp[rs + (q - rs + 1u) % wpr];          // word holding site x+32
    const uint32_t right = (a >> 1) | (nx << 31);              // +x neighbours of the 32 sites
    const uint32_t ps = q - q % wpp;                           // first word of the plane
    const uint32_t down = sp[ps + (q - ps + wpr) % wpp];       // +y neighbours
    uint32_t ux = a ^ right, uy = a ^ down;
    if (DIM == 3) {
      ux ^= st.bonds[q];
      uy ^= st.bonds[nwr + q];
      const uint32_t uz = a ^ sp[(q + wpp) % nwr] ^ st.bonds[2u * nwr + q]; // +z neighbours
      e += 2 * (int)__builtin_popcount(uz) - 32;
    }
    e += 2 * (int)(__builtin_popcount(ux) + __builtin_popcount(uy)) - 64;
    m += 32 - 2 * (int)__builtin_popcount(a);
  }
  e = wave_sum(e);
  m = wave_sum(m);
  if ((threadIdx.x & 63u) == 0u) {
    atomicAdd(&st.E[w], e);
    atomicAdd(&st.M[w], m);
  }
}

template <int DIM>
__global__ void k_recount(DevState st, Geometry G, uint32_t cur) {
  const uint32_t w = blockIdx.y;
  const uint32_t *sp = st.spins[cur] + (size_t)w * G.nwr;
  const uint32_t L = G.L;
  int e = 0, m = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < G.N; i += gridDim.x * blockDim.x) {
    const uint32_t x = i % L, y = (i / L) % L;
    const uint32_t bi = bit_at(sp, i);
    const uint32_t jx = i - x + (x + 1u == L ? 0u : x + 1u);
    const uint32_t jy = i - y * L + (y + 1u == L ? 0u : y + 1u) * L;
    uint32_t ux = bi ^ bit_at(sp, jx), uy = bi ^ bit_at(sp, jy);
    if (DIM == 3) {
      const uint32_t z = i / (L * L);
      const uint32_t jz = i - z * L * L + (z + 1u == L ? 0u : z + 1u) * L * L;
      const uint32_t nw = G.nwr;
      ux ^= bit_at(st.bonds, i);
      uy ^= bit_at(st.bonds + nw, i);
      const uint32_t uz = bi ^ bit_at(sp, jz) ^ bit_at(st.bonds + 2u * nw, i);
      e += 2 * (int)uz - 1; // bond energy -J s s = +1 if unsatisfied, -1 if satisfied
    }
    e += 2 * (int)(ux + uy) - 2;
    m += 1 - 2 * (int)bi;
  }
  e = wave_sum(e);
  m = wave_sum(m);
  if ((threadIdx.x & 63u) == 0u) {
    atomicAdd(&st.E[w], e);
    atomicAdd(&st.M[w], m);
  }
}

uint32_t ilog2(uint32_t v) {
  uint32_t r = 0;
  while ((1u << r) < v) ++r;
  return r;
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int DIM, int V>
hipError_t launch_tiled_v(const TiledArgs &a, uint32_t tiles, uint32_t R, uint32_t threads,
                          size_t lds, hipStream_t stream) {
  hipError_t err = allow_lds(k_tiled<DIM, V>, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_tiled<DIM, V>), dim3(tiles, R), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

template <int V>
hipError_t launch_tiled_n_v(const TiledArgs &a, uint32_t tiles, uint32_t R, uint32_t threads,
                            size_t lds, hipStream_t stream) {
  hipError_t err = allow_lds(k_tiled_n<V>, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_tiled_n<V>), dim3(tiles, R), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

template <int DIM, int V>
hipError_t launch_batch_sweep_v(const BatchInst *insts, const BatchItem *items, uint32_t n_items,
                                uint32_t W, uint32_t threads, uint32_t K, size_t lds,
                                hipStream_t stream) {
  hipError_t err = allow_lds(k_batch_sweep<DIM, V>, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_batch_sweep<DIM, V>), dim3(n_items), dim3(threads), lds, stream, insts,
                     items, W, K);
  return hipGetLastError();
}

template <int DIM, int V>
hipError_t launch_persist_v(PersistArgs &a, uint32_t R, uint32_t threads, size_t lds,
                            hipStream_t stream) {
  hipError_t err = allow_lds(k_persist<DIM, V>, lds);
  if (err != hipSuccess) return err;
  void *args[] = {&a};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_persist<DIM, V>), dim3(R),
                                    dim3(threads), args, (unsigned int)lds, stream);
}

template <int DIM, int V, int P>
hipError_t launch_persist_split_v(PersistArgs &a, uint32_t R, uint32_t threads, size_t lds,
                                  hipStream_t stream) {
  hipError_t err = allow_lds(k_persist_split<DIM, V, P>, lds);
  if (err != hipSuccess) return err;
  void *args[] = {&a};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_persist_split<DIM, V, P>),
                                    dim3(P * R), dim3(threads), args, (unsigned int)lds, stream);
}

// 2D split launch for V groups per item and 2, 4 or 8 parts.
template <int V>
hipError_t launch_persist_split_2d(PersistArgs &a, uint32_t R, uint32_t parts, uint32_t threads,
                                   size_t lds, hipStream_t stream) {
  return parts == 8   ? launch_persist_split_v<2, V, 8>(a, R, threads, lds, stream)
         : parts == 4 ? launch_persist_split_v<2, V, 4>(a, R, threads, lds, stream)
                      : launch_persist_split_v<2, V, 2>(a, R, threads, lds, stream);
}

// Groups per item of the split kernel: one item per thread in a colour-1 pass
// (a power of two, at most the groups of a row and kPersistSpan, 2D kNibbleSpan).
uint32_t split_span(const Geometry &g, uint32_t threads, uint32_t parts) {
  const uint32_t per = (g.L / parts) * g.rows * g.gpr / std::max<uint32_t>(threads, 1u);
  const uint32_t cap = std::min<uint32_t>(g.dim == 3 ? kPersistSpan : kNibbleSpan, g.gpr);
  uint32_t V = 1u;
  while (V * 2u <= per && V * 2u <= cap) V *= 2u;
  return V;
}

template <int V>
const void *split_fn_2d(uint32_t parts) {
  return parts == 8   ? reinterpret_cast<const void *>(k_persist_split<2, V, 8>)
         : parts == 4 ? reinterpret_cast<const void *>(k_persist_split<2, V, 4>)
                      : reinterpret_cast<const void *>(k_persist_split<2, V, 2>);
}

const void *split_fn(uint32_t dim, uint32_t V, uint32_t parts) {
  if (dim == 3)
    return V == 4   ? reinterpret_cast<const void *>(k_persist_split<3, 4, 2>)
           : V == 2 ? reinterpret_cast<const void *>(k_persist_split<3, 2, 2>)
                    : reinterpret_cast<const void *>(k_persist_split<3, 1, 2>);
  return V == 8 ? split_fn_2d<8>(parts) : V == 4 ? split_fn_2d<4>(parts)
       : V == 2 ? split_fn_2d<2>(parts) : split_fn_2d<1>(parts);
}

// Shape of the phased layout for a 2D lattice of side L (even).
struct PhasedShape {
  uint32_t Gmin, Gmax; // groups touched by the rows of phase 0 (fewest) and of the largest phase
  uint32_t S;          // LDS dwords per row
  uint32_t V;          // groups per interior span
  uint32_t nI, nE;     // interior spans and single-group items per row
  uint32_t lds_rows;   // LDS dword of the per-row table
  size_t lds;          // LDS bytes
};

PhasedShape phased_shape(const Geometry &g) {
  PhasedShape p;
  const uint32_t L = g.L;
  // row phases (y L) mod 8 are the multiples of gcd(L, 8) below 8
  const uint32_t step = (L & 7u) == 0u ? 8u : (L & 3u) == 0u ? 4u : 2u;
  const uint32_t phmax = step == 8u ? 0u : 8u - step;
  p.Gmin = (L + 7u) / 8u;
  p.Gmax = (phmax + L + 7u) / 8u;
  p.S = (p.Gmax + 3u) & ~3u;
  p.V = p.Gmin >= 6u ? 4u : 1u;
  p.nI = p.Gmin >= 2u ? (p.Gmin - 2u) / p.V : 0u;
  p.nE = p.Gmax - p.nI * p.V;
  p.lds_rows = (kPhasedLead + L * p.S + 4u + 3u) & ~3u;
  p.lds = (size_t)p.lds_rows * 4u + (size_t)L * 16u;
  return p;
}

template <int V>
hipError_t launch_phased_v(const PhasedArgs &a, uint32_t R, uint32_t threads, size_t lds,
                           hipStream_t stream) {
  hipError_t err = allow_lds(k_phased<V>, lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_phased<V>), dim3(1, R), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

template <int DIM, int V>
hipError_t launch_fused_v(const FusedArgs &a, uint32_t threads, size_t lds, hipStream_t stream) {
  const bool pf = (a.geo.R << a.lg_items) <= threads; // one item per thread at most
  hipError_t err = pf ? allow_lds(k_fused<DIM, V, true>, lds) : allow_lds(k_fused<DIM, V, false>, lds);
  if (err != hipSuccess) return err;
  if (pf) hipLaunchKernelGGL((k_fused<DIM, V, true>), dim3(1), dim3(threads), lds, stream, a);
  else hipLaunchKernelGGL((k_fused<DIM, V, false>), dim3(1), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

}  // namespace

size_t max_lds_bytes() { return 160u * 1024u - 1024u; }

size_t tiled_lds_bytes(const Geometry &g, uint32_t tile_planes, uint32_t halo) {
  if (g.phased) return phased_lds_bytes(g);
  const size_t np = (size_t)std::min(tile_planes, g.L) + 2u * halo;
  return np * g.plane / 2u * (g.dim == 3 ? 4u : 1u); // four bits per site; 3D: spins + 3 bond planes
}

size_t phased_lds_bytes(const Geometry &g) { return phased_shape(g).lds; }

size_t fused_lds_bytes(const Geometry &g) { return fused_layout(g.R, g.N, g.dim, 0u).total; }

size_t persist_lds_bytes(const Geometry &g, uint32_t parts) {
  if (parts >= 2u) {
    // L/parts + 4 staged planes of spins (and, 3D, three bond arrays), every
    // slot's thresholds; at least 96 KB, so that one part holds a compute
    // unit alone (all parts of a walker must advance at the same rate)
    const size_t need = (size_t)(g.L / parts + 4u) * g.plane / 2u * (g.dim == 3 ? 4u : 1u) +
                        (size_t)g.R * kClasses * 8u;
    return std::max<size_t>(need, 96u * 1024u);
  }
  return (size_t)g.N / 2u * (g.dim == 3 ? 4u : 1u) + (size_t)g.R * kClasses * 8u; // four bits per site
}

uint32_t persist_max_workgroups(const Geometry &g, uint32_t threads, uint32_t parts) {
  const uint32_t V = std::min<uint32_t>(kPersistSpan, g.gpr);
  const void *fn = parts >= 2u ? split_fn(g.dim, split_span(g, threads, parts), parts)
                 : g.dim == 3 ? (V == 4   ? reinterpret_cast<const void *>(k_persist<3, 4>)
                                 : V == 2 ? reinterpret_cast<const void *>(k_persist<3, 2>)
                                          : reinterpret_cast<const void *>(k_persist<3, 1>))
                 : V == 4 ? reinterpret_cast<const void *>(k_persist<2, 4>)
                 : V == 2 ? reinterpret_cast<const void *>(k_persist<2, 2>)
                          : reinterpret_cast<const void *>(k_persist<2, 1>);
  const size_t lds = persist_lds_bytes(g, parts);
  if (lds > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)threads, lds) != hipSuccess) return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return (uint32_t)(per_cu * cus);
}

hipError_t launch_init_spins(const DevState &st, const Geometry &g, const Keys &k, bool upload,
                             hipStream_t stream) {
  const uint64_t total = (uint64_t)g.nwr * g.R;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>((total + 255) / 256, 65535);
  hipLaunchKernelGGL(k_init_spins, dim3(blocks), dim3(256), 0, stream, st, g, k,
                     upload ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_init_bonds(const DevState &st, const Geometry &g, const Keys &k, bool upload,
                             hipStream_t stream) {
  const uint32_t blocks = std::min<uint32_t>((3u * (g.N >> 5) + 255u) / 256u, 65535u);
  hipLaunchKernelGGL(k_init_bonds, dim3(blocks), dim3(256), 0, stream, st, g, k,
                     upload ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_reset(const DevState &st, const Geometry &g, hipStream_t stream) {
  const uint32_t n = kMaxSweepsPerLaunch * g.R * 4u;
  const uint32_t hw = (uint32_t)split_halo_words(g);
  hipLaunchKernelGGL(k_reset, dim3((n + 255u) / 256u), dim3(256), 0, stream, st, g, hw);
  return hipGetLastError();
}

hipError_t launch_recount(const DevState &st, const Geometry &g, uint32_t cur,
                          hipStream_t stream) {
  if (g.L >= 32u && !g.phased) {
    // rows of whole packed words: one thread per word
    const uint32_t bx = std::min<uint32_t>(((g.N >> 5) + 255u) / 256u, 1024u);
    if (g.dim == 3)
      hipLaunchKernelGGL(k_recount_words<3>, dim3(bx, g.R), dim3(256), 0, stream, st, g, cur);
    else
      hipLaunchKernelGGL(k_recount_words<2>, dim3(bx, g.R), dim3(256), 0, stream, st, g, cur);
    return hipGetLastError();
  }
  const uint32_t bx = std::min<uint32_t>((g.N + 255u) / 256u, 1024u);
  if (g.dim == 3)
    hipLaunchKernelGGL(k_recount<3>, dim3(bx, g.R), dim3(256), 0, stream, st, g, cur);
  else
    hipLaunchKernelGGL(k_recount<2>, dim3(bx, g.R), dim3(256), 0, stream, st, g, cur);
  return hipGetLastError();
}

hipError_t launch_exchange(const DevState &st, const Geometry &g, const Keys &k, uint32_t e,
                           hipStream_t stream) {
  // one lane per pair of the step, all in flight together
  const uint32_t blocks = (g.R / 2u + 255u) / 256u;
  hipLaunchKernelGGL(k_exchange, dim3(blocks ? blocks : 1u), dim3(256), 0, stream, st, g.R, k, e);
  return hipGetLastError();
}

uint32_t span_groups(const Geometry &g) {
  return std::min<uint32_t>(g.gpr, g.dim == 3 ? 2u : 4u);
}

uint32_t batch_span(const Geometry &g) {
  return std::min<uint32_t>(g.gpr, g.dim == 3 ? 2u : kNibbleSpan);
}

hipError_t launch_tiled(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                        uint32_t tile_planes, uint32_t halo, uint32_t threads,
                        const Schedule &sch, hipStream_t stream) {
  if (halo == 0u && sch.do_exchange) {
    // whole replicas: the sweeps, then the exchange step as a launch of its own
    Schedule s2 = sch;
    s2.do_exchange = 0u;
    const hipError_t err = launch_tiled(st, g, k, cur, tile_planes, halo, threads, s2, stream);
    if (err != hipSuccess) return err;
    return launch_exchange(st, g, k, sch.ex_step, stream);
  }
  TiledArgs a;
  a.st = st;
  a.geo = g;
  a.key = k;
  a.sch = sch;
  a.H = std::min(tile_planes, g.L);
  a.halo = halo;
  a.src = st.spins[cur];
  a.dst = halo ? st.spins[cur ^ 1u] : st.spins[cur];
  if (g.phased) {
    // whole replicas only (the plan checks tile_planes >= L): rows of any even length
    const PhasedShape ps = phased_shape(g);
    PhasedArgs pa;
    pa.t = a;
    pa.t.H = g.L;
    pa.t.halo = 0u;
    pa.t.dst = st.spins[cur];
    pa.t.z2 = 8;
    pa.S = ps.S;
    pa.Gmax = ps.Gmax;
    pa.nI = ps.nI;
    pa.nE = ps.nE;
    pa.lds_rows = ps.lds_rows;
    return ps.V == 4 ? launch_phased_v<4>(pa, g.R, threads, ps.lds, stream)
                     : launch_phased_v<1>(pa, g.R, threads, ps.lds, stream);
  }
  const uint32_t V = span_groups(g);
  a.lg_L = ilog2(g.L);
  a.lg_spr = ilog2(g.gpr / V);
  a.lg_rows = ilog2(g.rows);
  a.z2 = g.dim == 3 ? 12 : 8;
  const uint32_t tiles = (g.L + a.H - 1u) / a.H;
  const size_t lds = tiled_lds_bytes(g, a.H, halo);
  if (g.dim == 3)
    return V == 2 ? launch_tiled_v<3, 2>(a, tiles, g.R, threads, lds, stream)
                  : launch_tiled_v<3, 1>(a, tiles, g.R, threads, lds, stream);
  // the nibble layout holds a group in one dword: up to kNibbleSpan groups per lane
  const uint32_t Vn = std::min<uint32_t>(kNibbleSpan, g.gpr);
  a.lg_spr = ilog2(g.gpr / Vn);
  return Vn == 8 ? launch_tiled_n_v<8>(a, tiles, g.R, threads, lds, stream)
       : Vn == 4 ? launch_tiled_n_v<4>(a, tiles, g.R, threads, lds, stream)
       : Vn == 2 ? launch_tiled_n_v<2>(a, tiles, g.R, threads, lds, stream)
                 : launch_tiled_n_v<1>(a, tiles, g.R, threads, lds, stream);
}

size_t lanes_lds_bytes(const Geometry &g) { return (size_t)g.R * (kClasses + 4u) * 4u; }

hipError_t launch_lanes(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                        const Schedule &sch, hipStream_t stream) {
  FusedArgs a;
  a.st = st;
  a.geo = g;
  a.key = k;
  a.sch = sch;
  a.spins = st.spins[cur];
  const uint32_t threads = (g.R + 63u) & ~63u;
  const size_t lds = lanes_lds_bytes(g);
  if (g.dim != 2 || (g.L != 8 && g.L != 16) || threads > (uint32_t)kMaxThreads)
    return hipErrorInvalidValue;
  hipError_t err = g.L == 8 ? allow_lds(k_lanes<8>, lds) : allow_lds(k_lanes<16>, lds);
  if (err != hipSuccess) return err;
  if (g.L == 8)
    hipLaunchKernelGGL(k_lanes<8>, dim3(1), dim3(threads), lds, stream, a);
  else
    hipLaunchKernelGGL(k_lanes<16>, dim3(1), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

size_t wave_lds_bytes(const Geometry &g) { return fused_layout(g.R, 0u, 2u, 0u).total; }

uint32_t wave_threads(const Geometry &g) { return (g.R * (g.N / 8u) + 63u) & ~63u; }

hipError_t launch_wave(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                       const Schedule &sch, hipStream_t stream) {
  const uint32_t threads = wave_threads(g);
  if (g.dim != 2 || (g.L != 8 && g.L != 16) || threads > (uint32_t)kMaxThreads)
    return hipErrorInvalidValue;
  FusedArgs a;
  a.st = st;
  a.geo = g;
  a.key = k;
  a.sch = sch;
  a.spins = st.spins[cur];
  a.lg_L = ilog2(g.L);
  a.lg_spr = 0u;
  a.lg_rows = 0u;
  a.lg_items = 0u;
  a.z2 = 8;
  // the swap-table rows go to LDS when they are small and fit beside the rest
  a.ntab = 0u;
  if ((size_t)st.swap_n * 8u <= 32u * 1024u &&
      fused_layout(g.R, 0u, 2u, st.swap_n).total <= max_lds_bytes())
    a.ntab = st.swap_n;
  const size_t lds = fused_layout(g.R, 0u, 2u, a.ntab).total;
  hipError_t err = g.L == 8 ? allow_lds(k_wave<8>, lds) : allow_lds(k_wave<16>, lds);
  if (err != hipSuccess) return err;
  if (g.L == 8)
    hipLaunchKernelGGL(k_wave<8>, dim3(1), dim3(threads), lds, stream, a);
  else
    hipLaunchKernelGGL(k_wave<16>, dim3(1), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

hipError_t launch_fused(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                        uint32_t threads, const Schedule &sch, hipStream_t stream) {
  FusedArgs a;
  a.st = st;
  a.geo = g;
  a.key = k;
  a.sch = sch;
  a.spins = st.spins[cur];
  const uint32_t V = span_groups(g);
  a.lg_L = ilog2(g.L);
  a.lg_spr = ilog2(g.gpr / V);
  a.lg_rows = ilog2(g.rows);
  a.lg_items = ilog2(g.N / (8u * V));
  a.z2 = g.dim == 3 ? 12 : 8;
  // the swap-table rows go to LDS when they are small and fit beside the rest
  a.ntab = 0u;
  if ((size_t)st.swap_n * 8u <= 32u * 1024u &&
      fused_layout(g.R, g.N, g.dim, st.swap_n).total <= max_lds_bytes())
    a.ntab = st.swap_n;
  const size_t lds = fused_layout(g.R, g.N, g.dim, a.ntab).total;
  if (g.dim == 3)
    return V == 2 ? launch_fused_v<3, 2>(a, threads, lds, stream)
                  : launch_fused_v<3, 1>(a, threads, lds, stream);
  return V == 4 ? launch_fused_v<2, 4>(a, threads, lds, stream)
       : V == 2 ? launch_fused_v<2, 2>(a, threads, lds, stream)
                : launch_fused_v<2, 1>(a, threads, lds, stream);
}

hipError_t launch_persist(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                          uint32_t threads, uint32_t parts, const Schedule &sch,
                          uint32_t spin_limit, hipStream_t stream) {
  PersistArgs a;
  a.st = st;
  a.geo = g;
  a.key = k;
  a.sch = sch;
  a.spins = st.spins[cur];
  a.lg_L = ilog2(g.L);
  a.lg_rows = ilog2(g.rows);
  a.z2 = g.dim == 3 ? 12 : 8;
  a.spin_limit = spin_limit;
  if (parts >= 2u) {
    if (parts > split_max_parts(g) || (parts & (parts - 1u)) || g.L / parts < 8u)
      return hipErrorInvalidValue;
    // the shares a part reads sit in consecutive lanes of one load round
    if (((4u * (g.plane / 32u)) & 63u) + 2u * (parts - 1u) > 64u) return hipErrorInvalidValue;
    const uint32_t V = split_span(g, threads, parts);
    a.lg_spr = ilog2(g.gpr / V);
    a.lg_ipp = g.dim == 3 ? a.lg_L + a.lg_spr : a.lg_spr;
    a.lg_items = 0u;
    const size_t lds = persist_lds_bytes(g, parts);
    if (g.dim == 3) {
      if (parts != 2u) return hipErrorInvalidValue;
      return V == 4   ? launch_persist_split_v<3, 4, 2>(a, g.R, threads, lds, stream)
             : V == 2 ? launch_persist_split_v<3, 2, 2>(a, g.R, threads, lds, stream)
                      : launch_persist_split_v<3, 1, 2>(a, g.R, threads, lds, stream);
    }
    return V == 8   ? launch_persist_split_2d<8>(a, g.R, parts, threads, lds, stream)
           : V == 4 ? launch_persist_split_2d<4>(a, g.R, parts, threads, lds, stream)
           : V == 2 ? launch_persist_split_2d<2>(a, g.R, parts, threads, lds, stream)
                    : launch_persist_split_2d<1>(a, g.R, parts, threads, lds, stream);
  }
  const uint32_t V = std::min<uint32_t>(kPersistSpan, g.gpr);
  a.lg_spr = ilog2(g.gpr / V);
  a.lg_items = ilog2(g.N / (8u * V));
  a.lg_ipp = 0u;
  const size_t lds = persist_lds_bytes(g, 1u);
  if (g.dim == 3)
    return V == 4   ? launch_persist_v<3, 4>(a, g.R, threads, lds, stream)
           : V == 2 ? launch_persist_v<3, 2>(a, g.R, threads, lds, stream)
                    : launch_persist_v<3, 1>(a, g.R, threads, lds, stream);
  return V == 4 ? launch_persist_v<2, 4>(a, g.R, threads, lds, stream)
       : V == 2 ? launch_persist_v<2, 2>(a, g.R, threads, lds, stream)
                : launch_persist_v<2, 1>(a, g.R, threads, lds, stream);
}

hipError_t launch_batch_tiled(const BatchInst *insts, const BatchTileItem *items, uint32_t n_items,
                              const Geometry &g, uint32_t H, uint32_t threads, uint32_t K,
                              hipStream_t stream) {
  if (n_items == 0) return hipSuccess;
  if (g.dim != 2 || K < 1 || K > kMaxSweepsPerLaunch || H < 1 || H > g.L ||
      (H < g.L && (2u * K > g.L / 2u || g.plane % 32u)))
    return hipErrorInvalidValue;
  const size_t lds = tiled_lds_bytes(g, H, H < g.L ? 2u * K : 0u);
  const uint32_t V = std::min<uint32_t>(kNibbleSpan, g.gpr);
  hipError_t err = hipSuccess;
  auto go = [&](auto kern) {
    if ((err = allow_lds(kern, lds)) != hipSuccess) return;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(threads), lds, stream, insts, items, H, K);
    err = hipGetLastError();
  };
  if (V == 8) go(k_batch_tiled<8>);
  else if (V == 4) go(k_batch_tiled<4>);
  else if (V == 2) go(k_batch_tiled<2>);
  else go(k_batch_tiled<1>);
  return err;
}

size_t batch_lds_bytes(const Geometry &g, uint32_t W) { return batch_layout(W, g.N, g.dim).total; }

hipError_t launch_batch_sweep(const BatchInst *insts, const BatchItem *items, uint32_t n_items,
                              const Geometry &g, uint32_t W, uint32_t threads, uint32_t K,
                              hipStream_t stream) {
  if (n_items == 0) return hipSuccess;
  const uint32_t V = batch_span(g);
  const size_t lds = batch_lds_bytes(g, W);
  if (g.dim == 3)
    return V == 2 ? launch_batch_sweep_v<3, 2>(insts, items, n_items, W, threads, K, lds, stream)
                  : launch_batch_sweep_v<3, 1>(insts, items, n_items, W, threads, K, lds, stream);
  if (V == 8) return launch_batch_sweep_v<2, 8>(insts, items, n_items, W, threads, K, lds, stream);
  return V == 4 ? launch_batch_sweep_v<2, 4>(insts, items, n_items, W, threads, K, lds, stream)
       : V == 2 ? launch_batch_sweep_v<2, 2>(insts, items, n_items, W, threads, K, lds, stream)
                : launch_batch_sweep_v<2, 1>(insts, items, n_items, W, threads, K, lds, stream);
}

hipError_t launch_batch_exchange(const BatchInst *insts, const uint2 *pairs, uint32_t n_pairs,
                                 uint32_t K, hipStream_t stream) {
  if (n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_exchange, dim3((n_pairs + 255u) / 256u), dim3(256), 0, stream, insts,
                     pairs, n_pairs, K);
  return hipGetLastError();
}

hipError_t launch_batch_advance(const BatchInst *insts, const uint32_t *list, uint32_t n, uint32_t K,
                                hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_advance, dim3((n + 255u) / 256u), dim3(256), 0, stream, insts, list, n,
                     K);
  return hipGetLastError();
}

hipError_t launch_batch_target(const BatchInst *insts, uint32_t n, uint32_t add, uint32_t every,
                               hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_target, dim3((n + 255u) / 256u), dim3(256), 0, stream, insts, n, add,
                     every);
  return hipGetLastError();
}

namespace {
__global__ void k_zero_words(uint64_t *p, size_t n) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
    p[q] = 0;
}
}  // namespace

hipError_t launch_zero(void *p, size_t bytes, hipStream_t stream) {
  const size_t n = bytes / 8u;
  if (n == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)std::min<size_t>((n + 255u) / 256u, 1024u);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, stream, (uint64_t *)p, n);
  return hipGetLastError();
}

hipError_t static_scratch(uint8_t **out) {
  static std::mutex mu;
  static std::vector<uint8_t *> addr; // per device, filled on first use
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if ((size_t)dev >= addr.size()) addr.resize((size_t)dev + 1u, nullptr);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || (uintptr_t)p % 256u) return hipErrorInvalidSymbol;
    addr[dev] = (uint8_t *)p;
  }
  *out = addr[dev];
  return hipSuccess;
}

}  // namespace ptmi
