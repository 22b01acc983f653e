// pt_kernels.hip -- gfx950 kernels of the parallel-tempering Metropolis library.
//
// Spin storage: one byte per site, 0 = up (s = +1), 1 = down (s = -1), so
// that the number of unsatisfied bonds of a site is a byte-wise sum of XORs.
// A lattice row of L sites is L/8 "groups" of 8 bytes; in every group the four
// sites of the colour being updated sit at byte positions off, off+2, off+4,
// off+6 (off = colour parity of the row), and they consume the four words of
// one Philox4x32-10 block whose counter is the group's index: the draw of site
// i is word (i/2) mod 4 of block (i/2)/4, as the method's draw mapping fixes.
//
// Work of one group (one lane): three (2D) or five (3D) 8-byte neighbour
// words plus one edge byte from LDS, a SWAR count of unsatisfied bonds per
// byte, one Philox block (18 64-bit multiplies + 20 three-way XORs), four
// LDS threshold lookups and compares, one 8-byte store, and the exact integer
// energy / magnetisation change of the accepted flips (dot4 bookkeeping).
//
// Kernels:
//   k_tiled<DIM>   grid (tiles, walkers).  A workgroup stages one tile of
//                  planes (rows in 2D, z-planes in 3D) plus halo planes of its
//                  walker in LDS and runs up to 8 sweeps on it.  With halo
//                  depth 2k for k sweeps the interior stays exact (every half
//                  sweep recomputes one plane less on each side with the same
//                  draws); tiles read one spin buffer and write the other.  A
//                  whole-replica tile (halo 0) updates in place.  The last
//                  workgroup to finish folds the per-sweep energy changes into
//                  E and M, writes the records, and runs the exchange step.
//   k_fused<DIM>   one workgroup holds every walker of a small system in LDS
//                  and runs sweeps, records and exchange steps without leaving
//                  the kernel.
//   k_exchange     one exchange step (slot permutation, no lattice copies).
//   k_init_*, k_reset, k_recount   initialisation.
#include "pt_internal.h"

#include <algorithm>

namespace ptmi {
namespace {

constexpr int kMaxThreads = 1024;

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
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

__device__ __forceinline__ uint2 lds_ld8(const uint8_t *p) {
  return *reinterpret_cast<const uint2 *>(p);
}
__device__ __forceinline__ void lds_st8(uint8_t *p, uint32_t lo, uint32_t hi) {
  *reinterpret_cast<uint2 *>(p) = make_uint2(lo, hi);
}

// Per-lane tallies of accepted flips: n = count, sb = sum of b (down spins
// flipped up), sc = sum of class index 8b+u.  Energy change of the tally:
// dE_int = 2z n - 4 (sc - 8 sb), magnetisation change dM = 4 sb - 2 n.
struct Tally {
  int n, sb, sc;
};

// Metropolis decision for the four colour sites of a group, given the centre
// word W, the per-byte unsatisfied-bond counts u (valid at the colour bytes),
// the colour offset and the four draws; returns the new centre word.
__device__ __forceinline__ uint2 decide(uint32_t wlo, uint32_t whi, uint32_t ulo, uint32_t uhi,
                                        uint32_t off, const Words &r, const uint32_t *thr,
                                        Tally &t) {
  const uint32_t sh = off << 3;
  const uint32_t wnlo = wlo >> sh, wnhi = whi >> sh;  // colour sites at bytes 0, 2
  const uint32_t clo = (wnlo << 3) | (ulo >> sh);     // class 8b+u per colour byte
  const uint32_t chi = (wnhi << 3) | (uhi >> sh);
  const uint32_t t0 = thr[clo & 15u];
  const uint32_t t1 = thr[(clo >> 16) & 15u];
  const uint32_t t2 = thr[chi & 15u];
  const uint32_t t3 = thr[(chi >> 16) & 15u];
  const uint32_t flo = (r.x <= t0 ? 1u : 0u) + (r.y <= t1 ? 0x10000u : 0u);
  const uint32_t fhi = (r.z <= t2 ? 1u : 0u) + (r.w <= t3 ? 0x10000u : 0u);
  t.n += (int)(__builtin_popcount(flo) + __builtin_popcount(fhi));
  t.sb = (int)__builtin_amdgcn_udot4(wnlo, flo, (uint32_t)t.sb, false);
  t.sb = (int)__builtin_amdgcn_udot4(wnhi, fhi, (uint32_t)t.sb, false);
  t.sc = (int)__builtin_amdgcn_udot4(clo, flo, (uint32_t)t.sc, false);
  t.sc = (int)__builtin_amdgcn_udot4(chi, fhi, (uint32_t)t.sc, false);
  return make_uint2(wlo ^ (flo << sh), whi ^ (fhi << sh));
}

// Byte index (within the row) of the edge byte the group needs: the site left
// of the group for off = 0, the site right of it for off = 1 (periodic).
__device__ __forceinline__ uint32_t edge_index(uint32_t g, uint32_t off, uint32_t L) {
  return off ? ((8u * g + 8u) & (L - 1u)) : ((8u * g + L - 1u) & (L - 1u));
}

// 2D Ising group update.  row/up/dn: LDS rows; g: group; off: colour offset.
__device__ __forceinline__ void group2d(uint8_t *row, const uint8_t *up, const uint8_t *dn,
                                        uint32_t g, uint32_t L, uint32_t off, const Words &r,
                                        const uint32_t *thr, Tally &t) {
  const uint2 W = lds_ld8(row + 8u * g);
  const uint2 U = lds_ld8(up + 8u * g);
  const uint2 D = lds_ld8(dn + 8u * g);
  const uint32_t e = row[edge_index(g, off, L)];
  const uint32_t e0 = off ? 0u : e, e1 = off ? e : 0u;
  const uint32_t llo = (W.x << 8) | e0;                       // left neighbours
  const uint32_t lhi = __builtin_amdgcn_alignbyte(W.y, W.x, 3);
  const uint32_t rlo = __builtin_amdgcn_alignbyte(W.y, W.x, 1); // right neighbours
  const uint32_t rhi = (W.y >> 8) | (e1 << 24);
  const uint32_t ulo = ((U.x ^ W.x) + (D.x ^ W.x)) + ((llo ^ W.x) + (rlo ^ W.x));
  const uint32_t uhi = ((U.y ^ W.y) + (D.y ^ W.y)) + ((lhi ^ W.y) + (rhi ^ W.y));
  const uint2 nw = decide(W.x, W.y, ulo, uhi, off, r, thr, t);
  lds_st8(row + 8u * g, nw.x, nw.y);
}

// 3D +-J EA group update.  Spin and bond planes share one LDS plane indexing:
// plane p of spins at sp + p*P, of x/y/z bonds at bx/by/bz + p*P.
__device__ __forceinline__ void group3d(uint8_t *sp, const uint8_t *bx, const uint8_t *by,
                                        const uint8_t *bz, uint32_t P, uint32_t pl, uint32_t pu,
                                        uint32_t pd, uint32_t y, uint32_t g, uint32_t L,
                                        uint32_t off, const Words &r, const uint32_t *thr,
                                        Tally &t) {
  const uint32_t yu = (y + L - 1u) & (L - 1u), yd = (y + 1u) & (L - 1u);
  const uint32_t o = pl * P + y * L + 8u * g;    // this group
  const uint32_t oyu = pl * P + yu * L + 8u * g; // row y-1
  const uint32_t oyd = pl * P + yd * L + 8u * g; // row y+1
  const uint32_t ozu = pu * P + y * L + 8u * g;  // plane z-1
  const uint32_t ozd = pd * P + y * L + 8u * g;  // plane z+1
  const uint2 W = lds_ld8(sp + o);
  const uint2 Sy0 = lds_ld8(sp + oyu), Sy1 = lds_ld8(sp + oyd);
  const uint2 Sz0 = lds_ld8(sp + ozu), Sz1 = lds_ld8(sp + ozd);
  const uint2 Jx = lds_ld8(bx + o);              // bond to x+1
  const uint2 Jy0 = lds_ld8(by + oyu), Jy1 = lds_ld8(by + o);
  const uint2 Jz0 = lds_ld8(bz + ozu), Jz1 = lds_ld8(bz + o);
  const uint32_t ei = pl * P + y * L + edge_index(g, off, L);
  const uint32_t e = sp[ei];
  const uint32_t ej = off ? 0u : (uint32_t)bx[ei]; // bond from the left edge site (off = 0)
  const uint32_t e0 = off ? 0u : e, e1 = off ? e : 0u;
  const uint32_t llo = (W.x << 8) | e0;
  const uint32_t lhi = __builtin_amdgcn_alignbyte(W.y, W.x, 3);
  const uint32_t rlo = __builtin_amdgcn_alignbyte(W.y, W.x, 1);
  const uint32_t rhi = (W.y >> 8) | (e1 << 24);
  const uint32_t jllo = (Jx.x << 8) | ej;         // bond to x-1 = Jx of the left site
  const uint32_t jlhi = __builtin_amdgcn_alignbyte(Jx.y, Jx.x, 3);
  const uint32_t ulo = (xor3(llo, W.x, jllo) + xor3(rlo, W.x, Jx.x)) +
                       (xor3(Sy0.x, W.x, Jy0.x) + xor3(Sy1.x, W.x, Jy1.x)) +
                       (xor3(Sz0.x, W.x, Jz0.x) + xor3(Sz1.x, W.x, Jz1.x));
  const uint32_t uhi = (xor3(lhi, W.y, jlhi) + xor3(rhi, W.y, Jx.y)) +
                       (xor3(Sy0.y, W.y, Jy0.y) + xor3(Sy1.y, W.y, Jy1.y)) +
                       (xor3(Sz0.y, W.y, Jz0.y) + xor3(Sz1.y, W.y, Jz1.y));
  const uint2 nw = decide(W.x, W.y, ulo, uhi, off, r, thr, t);
  lds_st8(sp + o, nw.x, nw.y);
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// One exchange step with parity e & 1 on the given walker/slot maps.
__device__ void exchange_step(const DevState &st, uint32_t R, uint32_t k0, uint32_t k1,
                              uint32_t e, const int32_t *E, uint32_t *walker_at,
                              uint32_t *slot_of, uint32_t tid, uint32_t nt) {
  for (uint32_t k = (e & 1u) + 2u * tid; k + 1u < R; k += 2u * nt) {
    const uint32_t a = walker_at[k], b = walker_at[k + 1u];
    const int32_t d = (E[a] - E[b]) / 4; // E_int differences are multiples of 4
    const int32_t D = (int32_t)st.swap_D[k];
    uint64_t T;
    if (d < -D)
      T = st.swap_sat[2u * k];
    else if (d > D)
      T = st.swap_sat[2u * k + 1u];
    else
      T = st.swap_tab[st.swap_off[k] + (uint32_t)(d + D)];
    const uint32_t r = philox(k, e, 0u, kPurposeSwap, k0, k1).x;
    st.att[k] += 1u;
    if ((uint64_t)r < T) {
      walker_at[k] = b;
      walker_at[k + 1u] = a;
      slot_of[a] = k + 1u;
      slot_of[b] = k;
      st.acc[k] += 1u;
    }
  }
}

struct TiledArgs {
  DevState st;
  Geometry geo;
  Keys key;
  Schedule sch;
  const uint8_t *src;
  uint8_t *dst;
  uint32_t H;      // interior planes per tile (last tile may be shorter)
  uint32_t halo;   // halo planes per side (0 = whole replica, in place)
  uint32_t lg_gpr; // log2(L/8)
  uint32_t lg_rows;
  int32_t z2;      // 2 * coordination number (8 in 2D, 12 in 3D)
};

template <int DIM>
__global__ __launch_bounds__(kMaxThreads) void k_tiled(TiledArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint32_t s_thr[kClasses];
  __shared__ int s_red[kMaxThreads / 64][2];
  __shared__ uint32_t s_last;

  const Geometry &G = a.geo;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t tile = blockIdx.x, w = blockIdx.y;
  const uint32_t L = G.L, P = G.plane;
  const uint32_t y0 = tile * a.H;
  const uint32_t Ht = min(a.H, L - y0);
  const uint32_t halo = a.halo;
  const uint32_t np = Ht + 2u * halo;                  // LDS planes
  const uint32_t base = (y0 + L - halo) & (L - 1u);   // global plane of LDS plane 0
  const uint32_t slot = a.st.slot_of[w];
  if (tid < kClasses) s_thr[tid] = a.st.flip_thr[slot * kClasses + tid];

  uint8_t *sp = smem;
  uint8_t *bx = smem + (size_t)np * P;
  uint8_t *by = bx + (size_t)np * P;
  uint8_t *bz = by + (size_t)np * P;

  // Stage planes [base, base+np) mod L of this walker (and the bonds) in LDS.
  {
    const uint32_t words = np * (P >> 3), nw = G.N >> 3, first = base * (P >> 3);
    const uint2 *src = reinterpret_cast<const uint2 *>(a.src + (size_t)w * G.N);
    for (uint32_t q = tid; q < words; q += nt)
      reinterpret_cast<uint2 *>(sp)[q] = src[(first + q) & (nw - 1u)];
    if (DIM == 3) {
      const uint2 *b = reinterpret_cast<const uint2 *>(a.st.bonds);
      for (uint32_t q = tid; q < words; q += nt) {
        const uint32_t gq = (first + q) & (nw - 1u);
        reinterpret_cast<uint2 *>(bx)[q] = b[gq];
        reinterpret_cast<uint2 *>(by)[q] = b[nw + gq];
        reinterpret_cast<uint2 *>(bz)[q] = b[2u * nw + gq];
      }
    }
  }
  __syncthreads();

  const uint32_t gmask = G.gpr - 1u, rmask = G.rows - 1u;
  const uint32_t shp = a.lg_gpr + a.lg_rows;
  Tally t = {0, 0, 0};
  for (uint32_t hs = 0; hs < 2u * a.sch.nsw; ++hs) {
    const uint32_t c = hs & 1u;
    const uint32_t s = a.sch.s0 + (hs >> 1);
    const uint32_t ext = halo ? (halo - 1u - hs) : 0u;
    const uint32_t plo = halo - ext;                 // computed LDS planes [plo, phi)
    const uint32_t items = (Ht + 2u * ext) << shp;
    for (uint32_t q = tid; q < items; q += nt) {
      const uint32_t g = q & gmask;
      const uint32_t y = (q >> a.lg_gpr) & rmask;
      const uint32_t pl = plo + (q >> shp);
      const uint32_t pu = (pl == 0u) ? np - 1u : pl - 1u;
      const uint32_t pd = (pl + 1u == np) ? 0u : pl + 1u;
      const uint32_t gp = (base + pl) & (L - 1u);   // global plane coordinate
      const uint32_t off = (c + gp + (DIM == 3 ? y : 0u)) & 1u;
      const uint32_t ctr0 = ((gp << a.lg_rows) + y) * G.gpr + g;
      const Words r = philox(ctr0, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
      Tally tg = {0, 0, 0};
      if (DIM == 2)
        group2d(sp + pl * P, sp + pu * P, sp + pd * P, g, L, off, r, s_thr, tg);
      else
        group3d(sp, bx, by, bz, P, pl, pu, pd, y, g, L, off, r, s_thr, tg);
      if (pl >= halo && pl < halo + Ht) {
        t.n += tg.n;
        t.sb += tg.sb;
        t.sc += tg.sc;
      }
    }
    if (c == 1u) {
      int dE = a.z2 * t.n - 4 * (t.sc - 8 * t.sb);
      int dM = 4 * t.sb - 2 * t.n;
      t = {0, 0, 0};
      dE = wave_sum(dE);
      dM = wave_sum(dM);
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

  // Write the interior planes back (contiguous in global memory).
  {
    const uint32_t words = Ht * (P >> 3);
    uint2 *dst = reinterpret_cast<uint2 *>(a.dst + (size_t)w * G.N + (size_t)y0 * P);
    const uint2 *lsrc = reinterpret_cast<const uint2 *>(sp + (size_t)halo * P);
    for (uint32_t q = tid; q < words; q += nt) dst[q] = lsrc[q];
  }

  // The last workgroup to arrive folds the sweep results, records, exchanges.
  __syncthreads();
  if (tid == 0u) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); // publish this workgroup's tallies
    const uint32_t total = gridDim.x * gridDim.y;
    const uint32_t prev =
        __hip_atomic_fetch_add(a.st.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev + 1u == total) ? 1u : 0u;
  }
  __syncthreads();
  if (!s_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

  const uint32_t R = G.R;
  uint32_t rec = a.sch.rec_base;
  for (uint32_t j = 0; j < a.sch.nsw; ++j) {
    for (uint32_t v = tid; v < R; v += nt) {
      int32_t *acc = a.st.acc3 + ((size_t)j * R + v) * 4u;
      const int32_t dE = __hip_atomic_load(acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int32_t dM = __hip_atomic_load(acc + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(acc, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(acc + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a.st.E[v] += dE;
      a.st.M[v] += dM;
    }
    __syncthreads();
    const uint32_t s = a.sch.s0 + j;
    if (a.sch.record_every && (s + 1u) % a.sch.record_every == 0u) {
      for (uint32_t k = tid; k < R; k += nt) {
        const uint32_t v = a.st.walker_at[k];
        a.st.E_series[(size_t)rec * R + k] = a.st.E[v];
        a.st.M_series[(size_t)rec * R + k] = a.st.M[v];
      }
      ++rec;
    }
  }
  if (a.sch.do_exchange) {
    __syncthreads();
    exchange_step(a.st, R, a.key.k0, a.key.k1, a.sch.ex_step, a.st.E, a.st.walker_at,
                  a.st.slot_of, tid, nt);
  }
  __syncthreads();
  if (tid == 0u) __hip_atomic_store(a.st.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct FusedArgs {
  DevState st;
  Geometry geo;
  Keys key;
  Schedule sch;
  uint8_t *spins;  // in place
  uint32_t lg_gpr, lg_rows, lg_items; // log2(L/8), log2(rows), log2(N/8)
  int32_t z2;
};

// LDS layout of the fused kernel.
struct FusedLayout {
  uint32_t thr, wat, sof, E, M, acc, spins, bonds, total;
};
__host__ __device__ inline FusedLayout fused_layout(uint32_t R, uint32_t N, uint32_t dim) {
  FusedLayout f;
  f.thr = 0;
  f.wat = f.thr + R * kClasses * 4u;
  f.sof = f.wat + R * 4u;
  f.E = f.sof + R * 4u;
  f.M = f.E + R * 4u;
  f.acc = f.M + R * 4u;
  f.spins = (f.acc + R * 8u + 15u) & ~15u;
  f.bonds = f.spins + R * N;
  f.total = f.bonds + (dim == 3 ? 3u * N : 0u);
  return f;
}

template <int DIM>
__global__ __launch_bounds__(kMaxThreads) void k_fused(FusedArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const Geometry &G = a.geo;
  const uint32_t R = G.R, N = G.N, L = G.L, P = G.plane;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const FusedLayout F = fused_layout(R, N, DIM);
  uint32_t *thr = reinterpret_cast<uint32_t *>(smem + F.thr);
  uint32_t *wat = reinterpret_cast<uint32_t *>(smem + F.wat);
  uint32_t *sof = reinterpret_cast<uint32_t *>(smem + F.sof);
  int32_t *E = reinterpret_cast<int32_t *>(smem + F.E);
  int32_t *M = reinterpret_cast<int32_t *>(smem + F.M);
  int32_t *acc = reinterpret_cast<int32_t *>(smem + F.acc);
  uint8_t *sp = smem + F.spins;
  uint8_t *bx = smem + F.bonds, *by = bx + N, *bz = by + N;

  for (uint32_t q = tid; q < R * kClasses; q += nt) thr[q] = a.st.flip_thr[q];
  for (uint32_t q = tid; q < R; q += nt) {
    wat[q] = a.st.walker_at[q];
    sof[q] = a.st.slot_of[q];
    E[q] = a.st.E[q];
    M[q] = a.st.M[q];
    acc[2u * q] = 0;
    acc[2u * q + 1u] = 0;
  }
  {
    const uint32_t words = (R * N) >> 3;
    const uint2 *src = reinterpret_cast<const uint2 *>(a.spins);
    for (uint32_t q = tid; q < words; q += nt) reinterpret_cast<uint2 *>(sp)[q] = src[q];
    if (DIM == 3) {
      const uint2 *b = reinterpret_cast<const uint2 *>(a.st.bonds);
      for (uint32_t q = tid; q < (3u * N) >> 3; q += nt) reinterpret_cast<uint2 *>(bx)[q] = b[q];
    }
  }
  __syncthreads();

  const uint32_t gmask = G.gpr - 1u, rmask = G.rows - 1u, imask = (N >> 3) - 1u;
  const uint32_t shp = a.lg_gpr + a.lg_rows;
  const uint32_t items = R << a.lg_items;
  uint32_t rec = a.sch.rec_base, e = a.sch.ex_step;
  for (uint32_t j = 0; j < a.sch.nsw; ++j) {
    const uint32_t s = a.sch.s0 + j;
    for (uint32_t c = 0; c < 2u; ++c) {
      uint32_t cur = 0xFFFFFFFFu;
      Tally t = {0, 0, 0};
      for (uint32_t q = tid; q < items; q += nt) {
        const uint32_t w = q >> a.lg_items;
        const uint32_t li = q & imask;
        if (w != cur) {
          if (cur != 0xFFFFFFFFu) {
            atomicAdd(&acc[2u * cur], a.z2 * t.n - 4 * (t.sc - 8 * t.sb));
            atomicAdd(&acc[2u * cur + 1u], 4 * t.sb - 2 * t.n);
          }
          cur = w;
          t = {0, 0, 0};
        }
        const uint32_t g = li & gmask;
        const uint32_t y = (li >> a.lg_gpr) & rmask;
        const uint32_t pl = li >> shp;
        const uint32_t pu = (pl + L - 1u) & (L - 1u);
        const uint32_t pd = (pl + 1u) & (L - 1u);
        const uint32_t off = (c + pl + (DIM == 3 ? y : 0u)) & 1u;
        const uint32_t slot = sof[w];
        const uint32_t ctr0 = ((pl << a.lg_rows) + y) * G.gpr + g;
        const Words r = philox(ctr0, s, slot, c | kPurposeFlip, a.key.k0, a.key.k1);
        uint8_t *wsp = sp + (size_t)w * N;
        if (DIM == 2)
          group2d(wsp + pl * P, wsp + pu * P, wsp + pd * P, g, L, off, r, thr + slot * kClasses, t);
        else
          group3d(wsp, bx, by, bz, P, pl, pu, pd, y, g, L, off, r, thr + slot * kClasses, t);
      }
      if (cur != 0xFFFFFFFFu) {
        atomicAdd(&acc[2u * cur], a.z2 * t.n - 4 * (t.sc - 8 * t.sb));
        atomicAdd(&acc[2u * cur + 1u], 4 * t.sb - 2 * t.n);
      }
      __syncthreads();
    }
    for (uint32_t v = tid; v < R; v += nt) {
      E[v] += acc[2u * v];
      M[v] += acc[2u * v + 1u];
      acc[2u * v] = 0;
      acc[2u * v + 1u] = 0;
    }
    __syncthreads();
    if (a.sch.record_every && (s + 1u) % a.sch.record_every == 0u) {
      for (uint32_t k = tid; k < R; k += nt) {
        a.st.E_series[(size_t)rec * R + k] = E[wat[k]];
        a.st.M_series[(size_t)rec * R + k] = M[wat[k]];
      }
      ++rec;
    }
    __syncthreads(); // records read the maps before the exchange rewrites them
    if (a.sch.exchange_every && (s + 1u) % a.sch.exchange_every == 0u) {
      exchange_step(a.st, R, a.key.k0, a.key.k1, e, E, wat, sof, tid, nt);
      ++e;
    }
    __syncthreads();
  }

  {
    const uint32_t words = (R * N) >> 3;
    uint2 *dst = reinterpret_cast<uint2 *>(a.spins);
    for (uint32_t q = tid; q < words; q += nt) dst[q] = reinterpret_cast<const uint2 *>(sp)[q];
  }
  for (uint32_t q = tid; q < R; q += nt) {
    a.st.walker_at[q] = wat[q];
    a.st.slot_of[q] = sof[q];
    a.st.E[q] = E[q];
    a.st.M[q] = M[q];
  }
}

__global__ void k_exchange(DevState st, uint32_t R, Keys key, uint32_t e) {
  exchange_step(st, R, key.k0, key.k1, e, st.E, st.walker_at, st.slot_of, threadIdx.x,
                blockDim.x);
}

// Initial spins: site i of walker w takes word i mod 4 of block (i/4, w, 0, spin
// purpose); top bit set = down.  upload: convert caller-provided +-1 bytes.
__global__ void k_init_spins(DevState st, Geometry G, Keys key, uint32_t upload) {
  const uint32_t quads = G.N >> 2;
  const uint64_t total = (uint64_t)quads * G.R;
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < total;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t w = (uint32_t)(q / quads), i4 = (uint32_t)(q % quads);
    uint32_t out;
    if (upload) {
      const uint32_t v = reinterpret_cast<const uint32_t *>(st.staging)[q];
      out = (v >> 7) & 0x01010101u; // sign bit of each +-1 byte
    } else {
      const Words r = philox(i4, w, 0u, kPurposeSpin, key.k0, key.k1);
      out = (r.x >> 31) | ((r.y >> 31) << 8) | ((r.z >> 31) << 16) | ((r.w >> 31) << 24);
    }
    reinterpret_cast<uint32_t *>(st.spins[0])[q] = out;
  }
}

// EA couplings: bond b = 3 i + d takes word b mod 4 of block (b/4, 0, 0, bond purpose).
__global__ void k_init_bonds(DevState st, Geometry G, Keys key, uint32_t upload) {
  const uint32_t total = 3u * G.N;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    const uint32_t d = q / G.N, i = q % G.N;
    uint8_t v;
    if (upload) {
      v = (uint8_t)(((uint32_t)st.staging[q] >> 7) & 1u);
    } else {
      const uint32_t b = 3u * i + d;
      const Words r = philox(b >> 2, 0u, 0u, kPurposeBond, key.b0, key.k1);
      const uint32_t word = (b & 3u) == 0 ? r.x : (b & 3u) == 1 ? r.y : (b & 3u) == 2 ? r.z : r.w;
      v = (uint8_t)(word >> 31);
    }
    st.bonds[q] = v;
  }
}

__global__ void k_reset(DevState st, Geometry G) {
  const uint32_t R = G.R;
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
}

// Full recount of E_int and M of every walker from spin buffer cur.
template <int DIM>
__global__ void k_recount(DevState st, Geometry G, uint32_t cur) {
  const uint32_t w = blockIdx.y;
  const uint8_t *sp = st.spins[cur] + (size_t)w * G.N;
  const uint32_t L = G.L;
  int e = 0, m = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < G.N; i += gridDim.x * blockDim.x) {
    const uint32_t x = i & (L - 1u), y = (i / L) & (L - 1u);
    const uint32_t bi = sp[i];
    const uint32_t jx = i - x + ((x + 1u) & (L - 1u));
    const uint32_t jy = i - y * L + ((y + 1u) & (L - 1u)) * L;
    uint32_t ux = bi ^ sp[jx], uy = bi ^ sp[jy];
    if (DIM == 3) {
      const uint32_t z = i / (L * L);
      const uint32_t jz = i - z * L * L + ((z + 1u) & (L - 1u)) * L * L;
      ux ^= st.bonds[i];
      uy ^= st.bonds[G.N + i];
      const uint32_t uz = bi ^ sp[jz] ^ st.bonds[2u * G.N + i];
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

}  // namespace

size_t max_lds_bytes() { return 160u * 1024u - 1024u; }

size_t tiled_lds_bytes(const Geometry &g, uint32_t tile_planes, uint32_t halo) {
  const size_t np = (size_t)std::min(tile_planes, g.L) + 2u * halo;
  return np * g.plane * (g.dim == 3 ? 4u : 1u);
}

size_t fused_lds_bytes(const Geometry &g) { return fused_layout(g.R, g.N, g.dim).total; }

hipError_t launch_init_spins(const DevState &st, const Geometry &g, const Keys &k, bool upload,
                             hipStream_t stream) {
  const uint64_t total = (uint64_t)(g.N >> 2) * g.R;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>((total + 255) / 256, 65535);
  hipLaunchKernelGGL(k_init_spins, dim3(blocks), dim3(256), 0, stream, st, g, k,
                     upload ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_init_bonds(const DevState &st, const Geometry &g, const Keys &k, bool upload,
                             hipStream_t stream) {
  const uint32_t blocks = std::min<uint32_t>((3u * g.N + 255u) / 256u, 65535u);
  hipLaunchKernelGGL(k_init_bonds, dim3(blocks), dim3(256), 0, stream, st, g, k,
                     upload ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_reset(const DevState &st, const Geometry &g, hipStream_t stream) {
  const uint32_t n = kMaxSweepsPerLaunch * g.R * 4u;
  hipLaunchKernelGGL(k_reset, dim3((n + 255u) / 256u), dim3(256), 0, stream, st, g);
  return hipGetLastError();
}

hipError_t launch_recount(const DevState &st, const Geometry &g, uint32_t cur,
                          hipStream_t stream) {
  const uint32_t bx = std::min<uint32_t>((g.N + 255u) / 256u, 1024u);
  if (g.dim == 3)
    hipLaunchKernelGGL(k_recount<3>, dim3(bx, g.R), dim3(256), 0, stream, st, g, cur);
  else
    hipLaunchKernelGGL(k_recount<2>, dim3(bx, g.R), dim3(256), 0, stream, st, g, cur);
  return hipGetLastError();
}

hipError_t launch_exchange(const DevState &st, const Geometry &g, const Keys &k, uint32_t e,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_exchange, dim3(1), dim3(256), 0, stream, st, g.R, k, e);
  return hipGetLastError();
}

hipError_t launch_tiled(const DevState &st, const Geometry &g, const Keys &k, uint32_t cur,
                        uint32_t tile_planes, uint32_t halo, uint32_t threads,
                        const Schedule &sch, hipStream_t stream) {
  TiledArgs a;
  a.st = st;
  a.geo = g;
  a.key = k;
  a.sch = sch;
  a.H = std::min(tile_planes, g.L);
  a.halo = halo;
  a.src = st.spins[cur];
  a.dst = halo ? st.spins[cur ^ 1u] : st.spins[cur];
  a.lg_gpr = ilog2(g.gpr);
  a.lg_rows = ilog2(g.rows);
  a.z2 = g.dim == 3 ? 12 : 8;
  const uint32_t tiles = (g.L + a.H - 1u) / a.H;
  const size_t lds = tiled_lds_bytes(g, a.H, halo);
  hipError_t err;
  if (g.dim == 3) {
    if ((err = allow_lds(k_tiled<3>, lds)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_tiled<3>, dim3(tiles, g.R), dim3(threads), lds, stream, a);
  } else {
    if ((err = allow_lds(k_tiled<2>, lds)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_tiled<2>, dim3(tiles, g.R), dim3(threads), lds, stream, a);
  }
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
  a.lg_gpr = ilog2(g.gpr);
  a.lg_rows = ilog2(g.rows);
  a.lg_items = ilog2(g.N >> 3);
  a.z2 = g.dim == 3 ? 12 : 8;
  const size_t lds = fused_lds_bytes(g);
  hipError_t err;
  if (g.dim == 3) {
    if ((err = allow_lds(k_fused<3>, lds)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_fused<3>, dim3(1), dim3(threads), lds, stream, a);
  } else {
    if ((err = allow_lds(k_fused<2>, lds)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_fused<2>, dim3(1), dim3(threads), lds, stream, a);
  }
  return hipGetLastError();
}

}  // namespace ptmi
