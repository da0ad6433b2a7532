// Matrix-core Hamming tile: kernels and launch templates, shared by the
// translation units that instantiate them (tile_mfma_w*.hip, one range of
// code lengths each, compiled in parallel). The design is described at the
// top of tile_mfma.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "wave_topk.h"

namespace bdg {
namespace mfma {


typedef int v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int kGroupKeys = 16; // keys one query can gain from one 16-code group

// 4 bits -> 4 bytes in {0, 1}: byte t = bit t. The multiplier places copies
// of the nibble at bit offsets 0, 7, 14, 21 (no two terms overlap), so bit t
// of the nibble lands at bit 8t.
__device__ __forceinline__ uint32_t spread_nibble(uint32_t nib) {
  return (nib * 0x00204081u) & 0x01010101u;
}

// 16 code bits -> 16 bytes of {0, 1} (0x01 for a set bit, 0x00 for a clear one).
__device__ __forceinline__ v4i expand_01(uint32_t h) {
  v4i r;
#pragma unroll
  for (int t = 0; t < 4; ++t) r[t] = (int)spread_nibble((h >> (4 * t)) & 15u);
  return r;
}

// 16 code bits -> 16 bytes of +-1 (0x01 for a set bit, 0xFF for a clear one).
__device__ __forceinline__ v4i expand_pm1(uint32_t h) {
  v4i r;
#pragma unroll
  for (int t = 0; t < 4; ++t)
    r[t] = (int)((spread_nibble((h >> (4 * t)) & 15u) * 0xFEu) ^ 0xFFFFFFFFu);
  return r;
}

// Operand bytes of code `row`, word s, lane quarter kq: +-1 (the queries) or
// {0, 1} (the candidate fragments).
__device__ __forceinline__ v4i code_chunk_pm1(const uint64_t* codes, uint32_t W, uint32_t row,
                                              uint32_t s, uint32_t kq) {
  const uint64_t w = codes[(size_t)row * W + s];
  return expand_pm1((uint32_t)(w >> (16 * kq)) & 0xFFFFu);
}
__device__ __forceinline__ v4i code_chunk_01(const uint64_t* codes, uint32_t W, uint32_t row,
                                             uint32_t s, uint32_t kq) {
  const uint64_t w = codes[(size_t)row * W + s];
  return expand_01((uint32_t)(w >> (16 * kq)) & 0xFFFFu);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work-group barrier for the stage ring. It emits no memory wait: each
// thread has already waited for its own stage copies (explicit vm-counter
// wait), and the reads of the buffer about to be overwritten have completed
// (their data fed the matrix cores). The signal fences keep the compiler
// from moving LDS accesses across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// s_waitcnt that waits for at most n outstanding vector-memory operations and
// nothing else (gfx9 encoding: vmcnt in bits 3:0 and 15:14).
#define BDG_WAIT_VMCNT(n) \
  __builtin_amdgcn_s_waitcnt(((n) & 15) | (((n) >> 4) << 14) | (7 << 4) | (15 << 8))

// One 16-byte-per-lane copy from global memory straight into LDS: lane l's
// 16 bytes land at LDS address lds + 16 l (lds is wave-uniform, in M0). It is
// written as inline assembly so that the compiler does not track it: its
// completion is waited for explicitly (vector-memory counter) and published
// to the other waves through the stage ring below. The instruction has no
// register destination.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"  // m0 is clobbered on purpose
__device__ __forceinline__ void dma16(const void* gptr, uint32_t lds) {
  asm volatile(
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %0, off"
      :
      : "v"(gptr), "s"(lds)
      : "memory", "m0");
}
#pragma clang diagnostic pop

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const lds_void*)p;
}

// Copy one stage (SV4 16-byte chunks, contiguous in HBM) into LDS with the
// NT threads of the work-group: every thread issues (SV4 + NT - 1) / NT copies
// (a wave past the end repeats whole 64-chunk pieces of the stage: the same
// bytes to the same place).
template <int SV4, int NT>
__device__ __forceinline__ void load_stage(const v4i* __restrict__ src, v4i* dst, uint32_t tid) {
  static_assert(NT % 64 == 0 && SV4 % 64 == 0, "whole waves");
  constexpr int LPS = (SV4 + NT - 1) / NT;
#pragma unroll
  for (int i = 0; i < LPS; ++i) {
    uint32_t v = i * NT + tid;
    if (SV4 % NT != 0 && v >= (uint32_t)SV4) v %= (uint32_t)SV4;
    dma16(src + v, __builtin_amdgcn_readfirstlane(lds_addr(dst + (v & ~63u))));
  }
}

// Copy one whole stage (SV4 16-byte chunks) with one wave.
template <int SV4>
__device__ __forceinline__ void load_stage_wave(const v4i* __restrict__ src, v4i* dst,
                                                uint32_t lane) {
  static_assert(SV4 % 64 == 0, "stage is whole wave copies");
  const uint32_t base = __builtin_amdgcn_readfirstlane(lds_addr(dst));
#pragma unroll
  for (int i = 0; i < SV4 / 64; ++i) dma16(src + i * 64 + lane, base + i * 1024);
}

// Pending keys of one query: KB slots in 4 sub-buffers of KB / 4, sub-buffer t
// owned by the lane of lane quarter t that holds the query in the MFMA output
// (lanes i, i + 16, i + 32, i + 48 for query i of a 16-query group), so a lane
// appends without coordinating with the others. cq[t] = keys in sub-buffer t.

// Merge the pending keys of one query into its list; returns the query's new
// threshold: the distance of the K-th key, or bits + 1 while the list is not
// full (a candidate enters only at a distance below it).
template <int NR, int KB>
__device__ __forceinline__ int flush_sub(uint32_t* list_q, const uint32_t* buf_q,
                                         uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t K, uint32_t lane, uint32_t IB, uint32_t bits) {
  constexpr int kBuf = KB, kSub = KB / 4;
  static_assert(kBuf <= 32 && kBuf % 4 == 0, "the pending keys of a query fit lanes 32..63");
  const uint32_t b = lane - 32u;  // slot of lane 32 + b
  const uint32_t t = b / kSub;
  const uint32_t ct = t == 0 ? c0 : (t == 1 ? c1 : (t == 2 ? c2 : c3));
  const uint32_t x =
      (lane >= 32u && b < (uint32_t)kBuf && b % kSub < ct) ? buf_q[b] : kKeyNone;
  uint32_t R[NR];
  load_list<NR>(list_q, R, K, lane);  // in flight together with the pending keys
  const uint32_t kth = merge_desc_with<NR>(list_q, R, wave_sort_upper32_desc(x, lane), K, lane);
  return kth == kKeyNone ? (int)bits + 1 : (int)(kth >> IB);
}

// One tile job: rows [row0, row0 + nrows) against columns [cb, ce). The lists
// of the rows live in out_idx/out_dist (row row0 + r at r * K); unless
// `fresh` they hold the merge of earlier column blocks. Keys and output
// indices are columns minus colbase (0: global indices; a shard's first row:
// shard-local indices). `bound` (row row0 + r at r), if not null, holds an
// upper bound on each row's final K-th distance (0xFFFF: none): while a list
// is not full only candidates at most the bound are admitted, which keeps the
// result exact and spares the admissions of far candidates seen early.
// `keys` (row row0 + r at r * K), if not null, holds the rows' running lists
// as keys in global memory instead of LDS (tile schedule 2): they are read and
// merged there, start empty when `fresh`, and are written to the output rows
// only by the job of the last column block (`last`).
struct TileJob {
  uint32_t row0, nrows, cb, ce, colbase;
  int fresh;
  uint32_t* out_idx;
  uint16_t* out_dist;
  const uint16_t* bound;
  uint32_t* keys = nullptr;
  int last = 1;
};

constexpr int kMaxWaves = 8;  // compute waves of a work-group, at most

// LDS of a tile besides the lists: the stage ring and its control words.
template <int SV4, int NST>
struct TileRing {
  v4i stage[NST][SV4];
  uint32_t landed[NST], claimed;
  uint32_t done[kMaxWaves];  // done[w] = stages compute wave w has read completely
  uint32_t published;        // with a producer: stages below this count have landed
};

// Whether every one of the NW compute waves has read all stages below `need`
// (one LDS read per lane for lanes < NW, wave-wide; the caller's lanes all
// take part).
template <int NW, int SV4, int NST>
__device__ __forceinline__ bool stages_read(TileRing<SV4, NST>& ring, uint32_t need, uint32_t lane) {
  static_assert(NW <= kMaxWaves, "done counters");
  const uint32_t d = lane < (uint32_t)NW
                         ? __hip_atomic_load(&ring.done[lane], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP)
                         : 0xFFFFFFFFu;
  return __ballot(d < need) == 0;
}

// The copy wave of a work-group with a producer (codes up to 512 bits): it
// streams the nst stages of the job into the ring and publishes them in order
// (published = number of stages whose copies are complete), keeping up to D
// stages in flight; a slot is refilled only after all NW compute waves have
// read its previous stage (their done counters). Before it sleeps on a slot
// it publishes everything it has issued, so that the compute waves never wait
// on a finished copy.
template <int SV4, int NST, int D, int NW>
__device__ __forceinline__ void produce_stages(TileRing<SV4, NST>& ring, const v4i* __restrict__ src0,
                                               uint32_t nst, uint32_t lane) {
  constexpr int LPS = SV4 / 64;  // copies per lane per stage
  static_assert(D >= 1 && D * LPS <= 63, "stages in flight exceed the vector-memory counter");
  uint32_t pub = 0;  // stages below pub are published
  auto publish_upto = [&](uint32_t end) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (end > pub && lane == 0)
      __hip_atomic_store(&ring.published, end, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    pub = end > pub ? end : pub;
  };
#pragma unroll 1
  for (uint32_t t = 0; t < nst; ++t) {
    const uint32_t slot = t % NST;
    if (t >= (uint32_t)NST) {
      const uint32_t need = t - NST + 1;  // the slot's previous stage is t - NST
      if (!stages_read<NW>(ring, need, lane)) {
        BDG_WAIT_VMCNT(0);
        publish_upto(t);
        while (!stages_read<NW>(ring, need, lane)) __builtin_amdgcn_s_sleep(1);
      }
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    load_stage_wave<SV4>(src0 + (size_t)t * SV4, ring.stage[slot], lane);
    if (t + 1 - pub > (uint32_t)D) {  // the oldest stage in flight must land first
      BDG_WAIT_VMCNT(D * LPS);
      publish_upto(t + 1 - D);
    }
  }
  BDG_WAIT_VMCNT(0);
  publish_upto(nst);
}

// The work of one work-group on one tile job; q0_wg = first job row of the
// work-group (the job's rows are split over work-groups of NW QW rows).
// RECT: rows and columns are different code sets (no column is a row's own
// pair), for the rectangular searches of the divide-and-conquer.
template <int W, int NR, int QG, int GPS, int NST, bool PROD, int NW, int KB, bool RECT = false,
          bool GL = false>
__device__ __forceinline__ void tile_body(const v4i* __restrict__ frags,
                                          const uint64_t* __restrict__ codes, uint32_t K,
                                          uint32_t bits, uint32_t IB, const TileJob& job,
                                          uint32_t q0_wg, TileRing<GPS * W * 64, NST>& ring,
                                          uint32_t* state) {
  // Groups contracted together: two where that brings more chains in flight
  // (QG <= 2) and the stage splits evenly (into an even number of units with
  // a producer, whose loop keeps the accumulator parity across stages).
  constexpr int U = (QG <= 2 && GPS % (PROD ? 4 : 2) == 0) ? 2 : 1;
  constexpr int NU = GPS / U;  // units per stage
  static_assert(!PROD || NU % 2 == 0, "the producer loop keeps accumulator parity across stages");
  constexpr int kBuf = KB, kSub = KB / 4;  // pending keys per query, per lane quarter
  constexpr int QW = 16 * QG;        // queries per wave
  constexpr int CT = 16 * GPS;       // codes per stage
  constexpr int SV4 = GPS * W * 64;  // 16-byte chunks per stage
  constexpr int kBufW = QW * kBuf + 64;  // + a discard slot per lane
  auto& stage = ring.stage;
  auto& ring_landed = ring.landed;
  auto& ring_claimed = ring.claimed;
  const uint32_t row0 = job.row0, nrows = job.nrows, cb = job.cb, ce = job.ce;
  const uint32_t colbase = job.colbase;
  const int fresh = job.fresh;
  constexpr bool rect = RECT;
  uint32_t* __restrict__ out_idx = job.out_idx;
  uint16_t* __restrict__ out_dist = job.out_dist;
  // lists in LDS [NW][QW][K] then the pending buffers [NW][kBufW]; with
  // GL the lists are in global memory (job.keys) and LDS holds the buffers
  uint32_t* lists = state;
  uint32_t* bufs = GL ? state : lists + NW * QW * K;

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const uint32_t i16 = lane & 15u;
  const uint32_t kq = lane >> 4;
  uint32_t* list_w = GL ? job.keys + (size_t)(q0_wg + wave * QW) * K : lists + wave * QW * K;
  uint32_t* buf_w = bufs + wave * kBufW;
  const uint32_t discard = QW * kBuf + lane;
  const uint32_t q0 = q0_wg + wave * QW;  // first job row of the wave
  const uint32_t imask = (1u << IB) - 1u;
  const uint32_t qlo = row0 + q0, qhi = row0 + q0 + QW;  // the wave's rows (as columns)

  const uint32_t cstart = cb & ~15u;
  const uint32_t nst = (ce - cstart + CT - 1) / CT;
  const v4i* src0 = frags + (size_t)(cstart / 16) * W * 64;
  // Stage ring control. The compute waves move through the stages
  // independently (a wave that merges lists does not hold the others back),
  // within the slack the ring allows: landed[b] = 1 + generation of the last
  // stage whose copy into slot b completed; done[w] counts the stages compute
  // wave w has read completely (one plain store per wave and stage; whoever
  // refills a slot checks all of them). With a producer wave, that wave does every
  // copy (produce_stages). Without one, claimed = next stage to be copied: the
  // first compute wave to reach a stage start claims the copy of the stage
  // NST - 1 ahead, issues it (the whole stage) once every wave has finished
  // the slot's previous stage, and publishes it at its next stage start.
  if (tid < NST) ring_landed[tid] = (!PROD && tid < NST - 1) ? 1u : 0u;  // prologue copies
  if (tid < kMaxWaves) ring.done[tid] = 0;
  if (tid == 0) ring.published = 0;
  if constexpr (PROD) {
    if (wave == NW) {
      lds_barrier();  // the ring words are initialised (pairs with the compute waves' barrier)
      constexpr int LPS = SV4 / 64;
      constexpr int DM = 63 / LPS;
      produce_stages<SV4, NST, (NST - 1 < DM ? NST - 1 : DM), NW>(ring, src0, nst, lane);
      return;
    }
  } else {
    if (tid == 0) ring_claimed = NST - 1;
#pragma unroll
    for (int p = 0; p < NST - 1; ++p)
      if ((uint32_t)p < nst) load_stage<SV4, NW * 64>(src0 + (size_t)p * SV4, stage[p], tid);
  }

  // Running lists of the wave's rows (the output rows, or with GL the keys in
  // global memory, hold the merge of the earlier column blocks unless this is
  // the first).
  if constexpr (GL) {
    if (fresh) {
      for (uint32_t p = lane; p < (uint32_t)(QW * K); p += kWave) {
        if (q0 + p / K >= nrows) break;  // rows past the job's end do not exist
        list_w[p] = kKeyNone;
      }
      BDG_WAIT_VMCNT(0);  // other lanes read these keys next
    }
  } else {
    for (uint32_t p = lane; p < (uint32_t)(QW * K); p += kWave) {
      const uint32_t q = p / K;
      uint32_t key = kKeyNone;
      if (!fresh && q0 + q < nrows) {
        const size_t o = (size_t)(q0 + q) * K + (p - q * K);
        const uint32_t j = out_idx[o];
        if (j != 0xFFFFFFFFu) key = ((uint32_t)out_dist[o] << IB) | j;
      }
      list_w[p] = key;
    }
  }
  wave_sync();

  // Query operands are +-1 bytes (s = 2q - 1), candidate operands {0, 1}
  // bytes (a), so the product is <s, a> = popc(q & a) - popc(~q & a) and
  // ham(q, a) = popc(q) - <s, a>. A candidate passes iff <s, a> + bias > 0
  // with the query's current bias thr - popc(q), applied when the unit is
  // filtered (so a threshold tightened since the contraction already counts).
  // ({0, 1} candidate bytes toggle far fewer multiplier bits than +-1 bytes,
  // which measurably raises the matrix cores' sustained rate.)
  v4i bq[QG][W];
  int biasQ[QG];
  int popcq[QG];
  int capB[QG];  // bias while the list is not full: bound + 1 - popc(q)
  uint32_t qrow[QG], csub[QG];
#pragma unroll
  for (int gq = 0; gq < QG; ++gq) {
    const uint32_t ql = q0 + 16 * gq + i16;
    const bool valid = ql < nrows;
    const uint32_t row = row0 + (valid ? ql : 0u);
    int pc = 0;
#pragma unroll
    for (int s = 0; s < W; ++s) {
      bq[gq][s] = code_chunk_pm1(codes, W, row, s, kq);
      pc += __popcll(codes[(size_t)row * W + s]);
    }
    int bias = -(int)bits - 1;  // absent row: acc <= popc(q) - bits - 1 < 0, never passes
    int cap = (int)bits + 1;
    if (valid) {
      if (job.bound) {
        const uint32_t b = job.bound[ql];
        if (b < bits) cap = (int)b + 1;
      }
      const uint32_t kth = list_w[(16 * gq + i16) * K + K - 1];
      // a full list holds only keys admitted under the bound: kth <= bound
      bias = (kth == kKeyNone ? cap : (int)(kth >> IB)) - pc;
    }
    biasQ[gq] = bias;
    capB[gq] = cap - pc;
    popcq[gq] = pc;
    qrow[gq] = row0 + ql;
    csub[gq] = 0;
  }

  if constexpr (PROD) {
    __syncthreads();  // ring init (pairs with the producer's barrier)
  } else {
    BDG_WAIT_VMCNT(0);  // prologue stage copies (all threads) and ring init
    __syncthreads();
  }

  // Flush every query of group gq whose lanes are flagged in m (a ballot).
  auto flush_group = [&](const int gq, uint64_t m) {
    uint32_t qm = (uint32_t)(m | (m >> 16) | (m >> 32) | (m >> 48)) & 0xFFFFu;
    wave_sync();
    while (qm) {
      const uint32_t i = __builtin_ctz(qm);
      qm &= qm - 1;
      const uint32_t qi = 16 * gq + i;
      const int thr = flush_sub<NR, KB>(
          list_w + qi * K, buf_w + qi * kBuf, __builtin_amdgcn_readlane(csub[gq], i),
          __builtin_amdgcn_readlane(csub[gq], 16 + i), __builtin_amdgcn_readlane(csub[gq], 32 + i),
          __builtin_amdgcn_readlane(csub[gq], 48 + i), K, lane, IB, bits);
      if (i16 == i) {
        biasQ[gq] = min(thr - popcq[gq], capB[gq]);
        csub[gq] = 0;
      }
      wave_sync();
    }
  };

  // Filter of the 16-code group starting at column cs: the largest
  // <s, a> + bias of a unit, and the appends of every candidate that beats its
  // query's threshold.
  auto max4b = [&](const v4i& acc, int gq) {
    return max(max(acc[0], acc[1]), max(acc[2], acc[3])) + biasQ[gq];
  };
  auto maxacc = [&](const v4i (&acc)[U][QG]) {
    int mx = max4b(acc[0][0], 0);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int gq = 0; gq < QG; ++gq) mx = max(mx, max4b(acc[u][gq], gq));
    return mx;
  };
  auto append = [&](const v4i (&acc)[QG], const uint32_t cs) {
    const uint32_t c0 = cs + 4 * kq;
    const bool edge = cs < cb || cs + 16 > ce;   // group crosses the column range
    const bool diag = !rect && cs < qhi && cs + 16 > qlo;  // group holds some of the wave's rows
#pragma unroll
    for (int gq = 0; gq < QG; ++gq) {
      if (!__any(max4b(acc[gq], gq) > 0)) continue;
      // Pass flags as sign bits: p_r = 1 iff <s, a>_r + bias > lim_r. lim_r =
      // 0, except (in the few groups on the column-range edge or holding the
      // wave's own rows) a column outside [cb, ce) or the query's own row
      // never passes (|<s, a> + bias| < 2^30, so the difference never wraps).
      int lim[4] = {0, 0, 0, 0};
      if (edge || diag) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t col = c0 + r;
          lim[r] = (col < cb || col >= ce || (!rect && col == qrow[gq])) ? 0x3FFFFFFF : 0;
        }
      }
      uint32_t pass[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) pass[r] = (uint32_t)(lim[r] - (acc[gq][r] + biasQ[gq])) >> 31;
      const uint32_t c = pass[0] + pass[1] + pass[2] + pass[3];
      const uint64_t over = __ballot(csub[gq] + c > (uint32_t)kSub);
      if (over) flush_group(gq, over);
      uint32_t pos = (16 * gq + i16) * kBuf + kq * kSub + csub[gq];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // popc(q) - <s, a> = ham, so this is ham << IB | column
        const uint32_t key = ((uint32_t)(popcq[gq] - acc[gq][r]) << IB) | (c0 + r - colbase);
        buf_w[pass[r] ? pos : discard] = key;
        pos += pass[r];
      }
      csub[gq] += c;
    }
  };

  // Units of U consecutive 16-code groups are contracted together: W layers
  // (one per 64-bit word) of U QG independent products. A scheduling fence
  // after each layer keeps a chain's consecutive products U QG issues apart
  // (never back to back), and `work(s)` places a share of the vector work
  // inside layer s. With U = 2 (two groups of 2 query tiles) four chains are
  // in flight, as many as with 4 query tiles.
  auto issue_with = [&](v4i (&acc)[U][QG], const v4i (&a)[U][W], auto&& work) {
#pragma unroll
    for (int s = 0; s < W; ++s) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int gq = 0; gq < QG; ++gq)
          acc[u][gq] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
              a[u][s], bq[gq][s], s == 0 ? v4i{0, 0, 0, 0} : acc[u][gq], 0, 0, 0);
      work(s);
      // without a producer, a fence per layer keeps each operand read after
      // the products that free its registers; with one, or with the lists in
      // global memory (two waves of 48 rows on a SIMD at 512 bits: 4.36
      // against 4.43 s), the compiler's own schedule of the reads was
      // measured faster
      if constexpr (!PROD && !GL) __builtin_amdgcn_sched_barrier(0);
    }
  };
  auto append_unit = [&](const v4i (&acc)[U][QG], const uint32_t cs) {
#pragma unroll
    for (int u = 0; u < U; ++u) append(acc[u], cs + 16 * u);
  };

  // Units are contracted in a ping-pong of accumulators: unit j is issued
  // before the filter of unit j - 1, so the matrix cores keep busy while the
  // vector ALUs test. A unit contracted before a merge tightened a threshold
  // just admits a superset; its keys use the bias it was contracted with. The
  // max-reduction of unit j - 1 is spread over the layers of unit j's
  // contraction (tile u QG + gq in layer (u QG + gq) % W), and so are the
  // operand reads of unit j + 1: layer s of unit j + 1 is read into the
  // registers layer s of unit j has just consumed, a whole unit ahead of its
  // use.
  v4i acc[2][U][QG];
  if constexpr (PROD) {
    // With a producer the unit stream runs across stage boundaries: the last
    // unit of stage st filters nothing new and reads the first unit of stage
    // st + 1 once that stage is known to have landed (a count read one unit
    // earlier, so the read never waits), and the first unit of a stage
    // filters the last unit of the previous one. The matrix cores then see no
    // gap at a stage start, except when the producer has fallen behind.
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int gq = 0; gq < QG; ++gq)
        acc[1][u][gq] = v4i{-(1 << 29), -(1 << 29), -(1 << 29), -(1 << 29)};  // nothing passes
    uint32_t avail = 0;  // stages known to have landed
    bool have = false;   // `a` already holds the operands of the stage's first unit
    v4i a[U][W];         // operands of the unit being contracted (then of the next)
    uint32_t slot = 0;   // st % NST
#pragma unroll 1
    for (uint32_t st = 0; st < nst; ++st) {
      const uint32_t nslot = slot + 1 == (uint32_t)NST ? 0u : slot + 1;
      const v4i* sb = stage[slot];
      const uint32_t cs0 = cstart + st * CT;
      if (!have) {
        while (st >= avail) {
          avail = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
              &ring.published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
          if (st >= avail) __builtin_amdgcn_s_sleep(1);
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int s = 0; s < W; ++s) a[u][s] = sb[(u * W + s) * 64 + lane];
      }
      // landed count, read now and looked at in the stage's last unit
      const uint32_t pubv = __hip_atomic_load(&ring.published, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
      bool pf = false;  // the next stage's first unit is read during the last unit
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        const v4i* nb = sb + (U * (j + 1)) * W * 64;  // operands of unit j + 1
        if (j + 1 == NU) {
          // every operand of the stage is in registers or on its way (this
          // wave's LDS reads complete in order, before the count below): the
          // slot can be reused
          // (every lane stores the same count: no lane mask to set up)
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
          __hip_atomic_store(&ring.done[wave], st + 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
          const uint32_t seen = __builtin_amdgcn_readfirstlane(pubv);
          avail = seen > avail ? seen : avail;
          pf = st + 1 < nst && st + 1 < avail;
          nb = stage[nslot];
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        __builtin_amdgcn_sched_barrier(0);
        v4i (&accP)[U][QG] = acc[(j + 1) & 1];  // the previous unit (stage st - 1's last for j = 0)
        int mx = -(1 << 29);
        issue_with(acc[j & 1], a, [&](int s) {
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int gq = 0; gq < QG; ++gq)
              if ((u * QG + gq) % W == s) mx = max(mx, max4b(accP[u][gq], gq));
          // (in the last unit these reads are made whether or not the next
          // stage has landed: reading a slot never disturbs the producer,
          // and operands read too early are read again at the stage start)
#pragma unroll
          for (int u = 0; u < U; ++u) a[u][s] = nb[(u * W + s) * 64 + lane];
        });
        if (__any(mx > 0)) append_unit(accP, cs0 + 16 * U * j - 16 * U);
      }
      have = pf;
      slot = nslot;
    }
    if (nst > 0) {
      if (__any(maxacc(acc[1]) > 0)) append_unit(acc[1], cstart + nst * CT - 16 * U);
    }
  } else {
  uint32_t pend = 0xFFFFFFFFu;  // stage this wave copies and has not published
#pragma unroll 1
  for (uint32_t st = 0; st < nst; ++st) {
    const uint32_t slot = st % NST;
    if (pend != 0xFFFFFFFFu) {  // publish the copy issued one stage ago
      BDG_WAIT_VMCNT(0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (lane == 0)
        __hip_atomic_store(&ring_landed[pend % NST], pend / NST + 1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
      pend = 0xFFFFFFFFu;
    }
    while (__hip_atomic_load(&ring_landed[slot], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP) < st / NST + 1)
      __builtin_amdgcn_s_sleep(1);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const uint32_t t = st + NST - 1;
    if (t < nst && __hip_atomic_load(&ring_claimed, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP) == t) {
      uint32_t won = 0;
      if (lane == 0) {
        uint32_t expect = t;
        won = __hip_atomic_compare_exchange_strong(&ring_claimed, &expect, t + 1,
                                                   __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP)
                  ? 1u
                  : 0u;
      }
      if (__builtin_amdgcn_readfirstlane(won)) {
        if (t >= (uint32_t)NST)
          while (!stages_read<NW>(ring, t - NST + 1, lane)) __builtin_amdgcn_s_sleep(1);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        load_stage_wave<SV4>(src0 + (size_t)t * SV4, stage[t % NST], lane);
        pend = t;
      }
    }
    const v4i* sb = stage[slot];
    const uint32_t cs0 = cstart + st * CT;
    v4i a[U][W];  // operands of the unit being contracted (then of the next)
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int s = 0; s < W; ++s) a[u][s] = sb[(u * W + s) * 64 + lane];
    if (NU % 2 == 0 && st > 0) {  // last unit of stage st - 1
      if (__any(maxacc(acc[1]) > 0)) append_unit(acc[1], cs0 - 16 * U);
    }
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      if (j + 1 == NU) {
        // every operand of the stage is in registers or on its way (this
        // wave's LDS reads complete in order, before the count below): the
        // slot can be reused
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (lane == 0)
          __hip_atomic_store(&ring.done[wave], st + 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      __builtin_amdgcn_sched_barrier(0);
      // operands of unit j + 1, layer s, once layer s of unit j is issued
      auto prefetch = [&](int s) {
        if (j + 1 < NU) {
#pragma unroll
          for (int u = 0; u < U; ++u) a[u][s] = sb[((U * (j + 1) + u) * W + s) * 64 + lane];
        }
      };
      if (j > 0) {
        v4i (&accP)[U][QG] = acc[(j - 1) & 1];
        int mx = -(1 << 29);
        issue_with(acc[j & 1], a, [&](int s) {
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int gq = 0; gq < QG; ++gq)
              if ((u * QG + gq) % W == s) mx = max(mx, max4b(accP[u][gq], gq));
          prefetch(s);
        });
        if (__any(mx > 0)) append_unit(accP, cs0 + 16 * U * (j - 1));
      } else {
        issue_with(acc[0], a, prefetch);
      }
    }
    if (NU % 2 != 0) {
      if (__any(maxacc(acc[(NU - 1) & 1]) > 0))
        append_unit(acc[(NU - 1) & 1], cs0 + 16 * U * (NU - 1));
    }
  }
  if (NU % 2 == 0 && nst > 0) {
    if (__any(maxacc(acc[1]) > 0)) append_unit(acc[1], cstart + nst * CT - 16 * U);
  }
  }
  BDG_WAIT_VMCNT(0);  // no stage copy of this wave is still in flight

  // Pending keys, then the lists back to the output rows (with GL only after
  // the last column block: until then the keys stay in global memory).
#pragma unroll
  for (int gq = 0; gq < QG; ++gq) {
    const uint64_t m = __ballot(csub[gq] > 0);
    if (m) flush_group(gq, m);
  }
  if constexpr (GL) {
    if (!job.last) return;
    BDG_WAIT_VMCNT(0);  // the merges' key stores, read back by other lanes
    wave_sync();
  }
  for (uint32_t p = lane; p < (uint32_t)(QW * K); p += kWave) {
    const uint32_t q = p / K;
    if (q0 + q >= nrows) break;
    const uint32_t key = list_w[p];
    const size_t o = (size_t)(q0 + q) * K + (p - q * K);
    out_idx[o] = key == kKeyNone ? 0xFFFFFFFFu : (key & imask);
    out_dist[o] = key == kKeyNone ? (uint16_t)0xFFFFu : (uint16_t)(key >> IB);
  }
}

// Launch shape per (code words W, list class NR: K <= 64 NR). Compute waves
// per work-group and 16-query groups per wave: lists of up to 64 keys take
// eight waves of 32 queries, two on each SIMD, so that one wave's filter,
// appends and merges overlap the other's products; longer lists, whose LDS
// leaves no room for that, four waves. Where the registers leave room for one
// more wave on a SIMD, an extra wave is the stage producer; otherwise the
// compute waves copy the stages themselves.
constexpr int waves_of_nr(int NR) { return NR == 1 ? 8 : 4; }
constexpr int qgroups_of_nr(int NR) { return NR == 1 ? 2 : (NR == 2 ? 3 : 1); }
constexpr bool use_producer(int W, int NR) { return NR == 1 ? W <= 4 : W <= 8; }
constexpr int threads_of(int W, int NR) {
  return (waves_of_nr(NR) + (use_producer(W, NR) ? 1 : 0)) * 64;
}
// 16-code groups per stage (even with a producer, so the ping-pong of
// accumulators runs across stage boundaries).
constexpr int stage_groups(int W, int NR) {
  return use_producer(W, NR) ? (W <= 4 ? 4 : 2) : (W <= 5 ? 4 : (W <= 8 ? 2 : 1));
}
// The LDS-list variants (template SC; every one computes the same graph): SC
// 0 = pending buffers of 32 keys per query (tile schedule 3); SC 1 = pending
// buffers of 16 keys per query, the LDS freed going to a deeper stage ring
// (more stages in flight, more frequent merges; tile schedule 1, built for
// codes of 128, 256 and 512 bits).
constexpr int kbuf_of(int SC) { return SC == 1 ? 16 : 32; }
constexpr bool sched_built(int W, int SC) { return SC == 0 || (W == 2 || W == 4 || W == 8); }
constexpr size_t state_bytes(int K, int qg, int nw, int kb = 32) {
  return (size_t)nw * ((size_t)16 * qg * K + (size_t)16 * qg * kb + 64) * 4;
}
// Stage slots: with a producer as many as the LDS left by lists of KC keys
// holds (at most 8); without, the previous fixed depths. KC is the list
// capacity class of K (kc_of): shorter lists leave room for more stages in
// flight, which the producer needs to cover the load latency of the stream.
constexpr int stages_of(int W, int NR, int KC, int SC = 0) {
  if (!use_producer(W, NR)) return NR == 2 ? 2 : 3;
  const size_t avail =
      160 * 1024 - state_bytes(KC, qgroups_of_nr(NR), waves_of_nr(NR), kbuf_of(SC)) - 256;
  const size_t n = avail / ((size_t)stage_groups(W, NR) * W * 1024);
  return n > 8 ? 8 : (int)n;
}

// One (row block, column block) tile per launch; work-group g takes rows
// [R g, R g + R) of the row block, R = NW QW.
template <int W, int NR, int QG, int GPS, int NST, int KB, bool RECT = false>
__global__ __launch_bounds__(threads_of(W, NR), 1) void knn_mfma_run_kernel(
    const v4i* __restrict__ frags, const uint64_t* __restrict__ codes, uint32_t K, uint32_t bits,
    uint32_t IB, TileJob job) {
  __shared__ TileRing<GPS * W * 64, NST> ring;
  extern __shared__ uint32_t state[];
  constexpr int NW = waves_of_nr(NR);
  tile_body<W, NR, QG, GPS, NST, use_producer(W, NR), NW, KB, RECT>(
      frags, codes, K, bits, IB, job, blockIdx.x * (NW * 16 * QG), ring, state);
}

// Many independent partitions in one persistent launch: every work-group
// takes work items (one shard's NW QW rows against all the shard's columns)
// from a shared counter until the list is exhausted. Items are ordered
// longest first, so the uneven shards balance over the CUs. GL: the lists are
// keys in the output index rows while the item runs (tile schedule 2).
template <int W, int NR, int QG, int GPS, int NST, int KB, int NW = waves_of_nr(NR),
          bool PR = use_producer(W, NR), bool GL = false>
__global__ __launch_bounds__((NW + (PR ? 1 : 0)) * 64, 1) void knn_mfma_batched_kernel(
    const v4i* __restrict__ frags, const uint64_t* __restrict__ codes, uint32_t K, uint32_t bits,
    uint32_t IB, const BatchItem* __restrict__ items, uint32_t nitems, uint32_t* counter,
    uint32_t* __restrict__ out_idx, uint16_t* __restrict__ out_dist,
    const uint16_t* __restrict__ bound, uint32_t bound_base) {
  __shared__ TileRing<GPS * W * 64, NST> ring;
  __shared__ uint32_t cur;
  extern __shared__ uint32_t state[];
  for (;;) {
    __syncthreads();  // every wave is done with the previous item
    if (threadIdx.x == 0) cur = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t it = cur;
    if (it >= nitems) break;  // work-group-uniform: every wave leaves
    const BatchItem b = items[it];
    TileJob job;
    job.row0 = b.row0;
    job.nrows = b.nrows;
    job.cb = b.lo;
    job.ce = b.hi;
    job.colbase = b.lo;
    job.fresh = 1;
    job.out_idx = out_idx + (size_t)b.row0 * K;
    job.out_dist = out_dist + (size_t)b.row0 * K;
    job.bound = bound ? bound + (b.row0 - bound_base) : nullptr;
    job.keys = GL ? job.out_idx : nullptr;
    job.last = 1;
    tile_body<W, NR, QG, GPS, NST, PR, NW, KB, false, GL>(frags, codes, K, bits, IB, job, 0, ring,
                                                          state);
  }
}

// Default bound on the polls of one dependency wait (each polls, then sleeps
// about 1,000 cycles): seconds, far beyond any item. The wait order makes the
// bound unreachable; it only guarantees that every wave exits. A caller can
// set a lower bound (a test forces the give-up path that way: every wave
// still exits normally and the stall flag is set).
constexpr uint32_t kSweepSpinLimit = 1u << 23;

// A whole build in one persistent launch (SweepArgs): every work-group takes
// items (row tile t, column block c) from a shared counter in the order
// c * ntiles + t, so that all work-groups stream the same column block at
// once (it stays in L2) and the launch ends on a tail of at most one item per
// work-group, where separate launches per block would each leave CUs idle in
// their last round. Item (t, c > 0) merges into the lists item (t, c - 1)
// wrote: it waits for progress[t] = c. That item was claimed earlier, by a
// work-group already running, and its own wait is on a still earlier item,
// down to a first-block item that waits for nothing, so every wait ends.
// GL: the running lists stay keys in the output index rows between column
// blocks (tile schedule 2), so the LDS holds no lists and NW compute waves of
// QG groups fit where the LDS-resident lists of the same K allow fewer.
template <int W, int NR, int QG, int GPS, int NST, int KB, int NW = waves_of_nr(NR),
          bool PR = use_producer(W, NR), bool GL = false>
__global__ __launch_bounds__((NW + (PR ? 1 : 0)) * 64, 1) void knn_mfma_sweep_kernel(
    const v4i* __restrict__ frags, const uint64_t* __restrict__ codes, uint32_t K, uint32_t bits,
    uint32_t IB, uint32_t row0, uint32_t nrows, uint32_t ncols, uint32_t col_block,
    uint32_t ntiles, uint32_t nitems, uint32_t* ctl, uint32_t* __restrict__ out_idx,
    uint16_t* __restrict__ out_dist, uint32_t spin_limit, const uint16_t* __restrict__ bound) {
  __shared__ TileRing<GPS * W * 64, NST> ring;
  __shared__ uint32_t cur;
  extern __shared__ uint32_t state[];
  constexpr uint32_t RT = NW * 16 * QG;  // rows per tile
  uint32_t* progress = ctl + 2;
  const uint32_t ncb = nitems / ntiles;
  for (;;) {
    __syncthreads();  // every wave is done with the previous item
    if (threadIdx.x == 0) cur = atomicAdd(ctl, 1u);
    __syncthreads();
    const uint32_t it = cur;
    if (it >= nitems) break;  // work-group-uniform: every wave leaves
    const uint32_t c = it / ntiles, t = it - c * ntiles;
    if (c > 0) {
      if (threadIdx.x == 0) {
        for (uint32_t spins = 0; __hip_atomic_load(&progress[t], __ATOMIC_ACQUIRE,
                                                   __HIP_MEMORY_SCOPE_AGENT) < c;) {
          if (++spins >= spin_limit) {
            __hip_atomic_store(&ctl[kSweepStallWord], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(16);
        }
      }
      __syncthreads();
      // the lists written by the previous item (on any XCD) are seen
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    TileJob job;
    job.row0 = row0 + t * RT;
    job.nrows = nrows - t * RT < RT ? nrows - t * RT : RT;
    job.cb = c * col_block;
    job.ce = ncols - job.cb < col_block ? ncols : job.cb + col_block;
    job.colbase = 0;
    job.fresh = c == 0;
    job.out_idx = out_idx + (size_t)t * RT * K;
    job.out_dist = out_dist + (size_t)t * RT * K;
    job.bound = bound ? bound + job.row0 : nullptr;
    job.keys = GL ? job.out_idx : nullptr;
    job.last = c + 1 == ncb;
    tile_body<W, NR, QG, GPS, NST, PR, NW, KB, false, GL>(frags, codes, K, bits, IB, job, 0, ring,
                                                          state);
    // the tile's lists are in the output rows: publish them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_store(&progress[t], c + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

namespace {
__global__ void zero_counter_kernel(uint32_t* counter) { *counter = 0; }
__global__ void zero_words_kernel(uint32_t* w, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) w[i] = 0;
}
}  // namespace

inline int nr_of(uint32_t K) { return K <= 64 ? 1 : (K <= 128 ? 2 : 4); }
// List capacity class: the stage ring of a launch is sized for lists of this
// many keys (at least K).
inline int kc_of(uint32_t K) {
  return K <= 32 ? 32 : (K <= 64 ? 64 : (K <= 112 ? 112 : (K <= 128 ? 128 : 256)));
}
inline int qg_of(uint32_t K) { return qgroups_of_nr(nr_of(K)); }
inline int nw_of(uint32_t K) { return waves_of_nr(nr_of(K)); }

inline size_t run_state_bytes(uint32_t K, int qg, int kb = 32) {
  return state_bytes((int)K, qg, nw_of(K), kb);
}

inline size_t run_lds_bytes(uint32_t W, uint32_t K) {
  const size_t stage = (size_t)stage_groups((int)W, nr_of(K)) * W * 1024;
  return stages_of((int)W, nr_of(K), kc_of(K)) * stage + run_state_bytes(K, qg_of(K));
}

template <int W, int NR, int KC>
inline hipError_t launch_run_w(const RunArgs& a, hipStream_t stream) {
  constexpr int QG = qgroups_of_nr(NR);
  constexpr int GPS = stage_groups(W, NR);
  constexpr int NST = stages_of(W, NR, KC);
  static_assert(NST >= 2, "stage ring needs two slots");
  // the rectangular variant exists for lists of up to 64 keys only
  auto kern = knn_mfma_run_kernel<W, NR, QG, GPS, NST, 32>;
  if (a.rect) {
    if constexpr (NR == 1)
      kern = knn_mfma_run_kernel<W, NR, QG, GPS, NST, 32, true>;
    else
      return hipErrorInvalidValue;
  }
  const size_t lds = run_state_bytes(a.K, QG);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const uint32_t rows_per_wg = waves_of_nr(NR) * 16 * QG;
  dim3 grid((a.nrows + rows_per_wg - 1) / rows_per_wg);
  TileJob job;
  job.row0 = a.row0;
  job.nrows = a.nrows;
  job.cb = a.cb;
  job.ce = a.ce;
  job.colbase = 0;
  job.fresh = a.fresh;
  job.out_idx = a.out_idx;
  job.out_dist = a.out_dist;
  job.bound = nullptr;
  hipLaunchKernelGGL(kern, grid, dim3(threads_of(W, NR)), lds, stream,
                     reinterpret_cast<const v4i*>(a.frags), a.codes, a.K, a.bits, a.idx_bits, job);
  return hipGetLastError();
}

template <int W, int NR, int KC, int SC>
inline hipError_t launch_batched_w(const BatchArgs& a, hipStream_t stream) {
  constexpr int QG = qgroups_of_nr(NR);
  constexpr int GPS = stage_groups(W, NR);
  constexpr int NST = stages_of(W, NR, KC, SC);
  static_assert(NST >= 2, "stage ring needs two slots");
  auto kern = knn_mfma_batched_kernel<W, NR, QG, GPS, NST, kbuf_of(SC)>;
  const size_t lds = run_state_bytes(a.K, QG, kbuf_of(SC));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, stream, a.counter);
  hipLaunchKernelGGL(kern, dim3(a.grid), dim3(threads_of(W, NR)), lds, stream,
                     reinterpret_cast<const v4i*>(a.frags), a.codes, a.K, a.bits, a.idx_bits,
                     a.items, a.nitems, a.counter, a.out_idx, a.out_dist, a.bound, a.bound_base);
  return hipGetLastError();
}

template <int W, int NR, int KC, int SC>
inline hipError_t launch_sweep_w(const SweepArgs& a, hipStream_t stream) {
  constexpr int QG = qgroups_of_nr(NR);
  constexpr int GPS = stage_groups(W, NR);
  constexpr int NST = stages_of(W, NR, KC, SC);
  static_assert(NST >= 2, "stage ring needs two slots");
  auto kern = knn_mfma_sweep_kernel<W, NR, QG, GPS, NST, kbuf_of(SC)>;
  const size_t lds = run_state_bytes(a.K, QG, kbuf_of(SC));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const uint32_t rt = waves_of_nr(NR) * 16 * QG;
  const uint32_t ntiles = (a.nrows + rt - 1) / rt;
  const uint32_t ncb = (a.ncols + a.col_block - 1) / a.col_block;
  if ((uint64_t)ntiles * ncb > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const uint32_t nitems = ntiles * ncb;
  const uint32_t words = ntiles + 2;
  hipLaunchKernelGGL(zero_words_kernel, dim3((words + 255) / 256), dim3(256), 0, stream, a.ctl,
                     words);
  const uint32_t grid = a.grid < nitems ? a.grid : nitems;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads_of(W, NR)), lds, stream,
                     reinterpret_cast<const v4i*>(a.frags), a.codes, a.K, a.bits, a.idx_bits,
                     a.row0, a.nrows, a.ncols, a.col_block, ntiles, nitems, a.ctl, a.out_idx,
                     a.out_dist, a.spin_limit ? a.spin_limit : kSweepSpinLimit, a.bound);
  return hipGetLastError();
}

// Tile schedule 2 (lists of up to 128 keys in global memory): eight compute
// waves of 48 rows (three 16-row groups), two on each SIMD, so every candidate
// operand read from the LDS feeds three products instead of two (at two groups
// the eight waves' operand reads alone fill the LDS bandwidth). The LDS holds
// the pending buffers (50 KB) and a stage ring of 64-code stages; where the
// registers leave room (codes of up to 256 bits) a ninth wave produces the
// stages, otherwise the compute waves copy them. Measured on 1M 256-bit codes,
// K = 64, and 4M 512-bit codes, K = 100: 163.6 -> 136.9 ms and 5.16 -> 4.46 s
// against the LDS lists of schedule 3; two groups per wave: 197.6 ms and
// 4.97 s; four: spills registers at 512 bits, 161.4 ms without a producer at
// 256. Stages of 32 codes in rings of five or six at 512 bits: 4.88 / 4.84 s.
constexpr int kGlQG = 3, kGlWaves = 8, kGlGroups = 4;
constexpr bool gl_built(int W) { return W == 2 || W == 4 || W == 8; }
constexpr bool gl_producer(int W) { return W <= 4; }
constexpr uint32_t kGlRows = kGlWaves * 16 * kGlQG;  // rows per tile
constexpr size_t gl_state_bytes() { return state_bytes(0, kGlQG, kGlWaves, 32); }
// Stage slots: three 32 KB stages without a producer (512 bits); with one, as
// many as the LDS holds up to five (measured: 5 slots 136.9 ms, 3 slots 138.5
// ms at 256 bits).
constexpr int gl_stages(int W) {
  if (!gl_producer(W)) return 3;
  const size_t n = (160 * 1024 - gl_state_bytes() - 256) / ((size_t)kGlGroups * W * 1024);
  return n > 5 ? 5 : (int)n;
}
constexpr int gl_threads(int W) { return (kGlWaves + (gl_producer(W) ? 1 : 0)) * 64; }

template <int W, int NR>
inline hipError_t launch_sweep_gl(const SweepArgs& a, hipStream_t stream) {
  constexpr int QG = kGlQG, NW = kGlWaves, GPS = kGlGroups, NST = gl_stages(W);
  constexpr bool PR = gl_producer(W);
  static_assert(NST >= 2 && sizeof(TileRing<GPS * W * 64, NST>) + gl_state_bytes() <= 160 * 1024,
                "stage ring and buffers fit the LDS");
  auto kern = knn_mfma_sweep_kernel<W, NR, QG, GPS, NST, 32, NW, PR, true>;
  const size_t lds = gl_state_bytes();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  constexpr uint32_t rt = kGlRows;
  const uint32_t ntiles = (a.nrows + rt - 1) / rt;
  const uint32_t ncb = (a.ncols + a.col_block - 1) / a.col_block;
  if ((uint64_t)ntiles * ncb > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const uint32_t nitems = ntiles * ncb;
  const uint32_t words = ntiles + 2;
  hipLaunchKernelGGL(zero_words_kernel, dim3((words + 255) / 256), dim3(256), 0, stream, a.ctl,
                     words);
  const uint32_t grid = a.grid < nitems ? a.grid : nitems;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(gl_threads(W)), lds, stream,
                     reinterpret_cast<const v4i*>(a.frags), a.codes, a.K, a.bits, a.idx_bits,
                     a.row0, a.nrows, a.ncols, a.col_block, ntiles, nitems, a.ctl, a.out_idx,
                     a.out_dist, a.spin_limit ? a.spin_limit : kSweepSpinLimit, a.bound);
  return hipGetLastError();
}

// Schedule 2 for batched plans: the same tile; an item covers all of its
// shard's columns, so its lists start empty and end in the output rows.
template <int W, int NR>
inline hipError_t launch_batched_gl(const BatchArgs& a, hipStream_t stream) {
  constexpr int QG = kGlQG, NW = kGlWaves, GPS = kGlGroups, NST = gl_stages(W);
  constexpr bool PR = gl_producer(W);
  auto kern = knn_mfma_batched_kernel<W, NR, QG, GPS, NST, 32, NW, PR, true>;
  const size_t lds = gl_state_bytes();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, stream, a.counter);
  hipLaunchKernelGGL(kern, dim3(a.grid), dim3(gl_threads(W)), lds, stream,
                     reinterpret_cast<const v4i*>(a.frags), a.codes, a.K, a.bits, a.idx_bits,
                     a.items, a.nitems, a.counter, a.out_idx, a.out_dist, a.bound, a.bound_base);
  return hipGetLastError();
}

template <int W, int SC>
inline hipError_t launch_sweep_sc(const SweepArgs& a, hipStream_t stream) {
  switch (kc_of(a.K)) {
    case 32: return launch_sweep_w<W, 1, 32, SC>(a, stream);
    case 64: return launch_sweep_w<W, 1, 64, SC>(a, stream);
    case 112: return launch_sweep_w<W, 2, 112, SC>(a, stream);
    case 128: return launch_sweep_w<W, 2, 128, SC>(a, stream);
    default: return launch_sweep_w<W, 4, 256, SC>(a, stream);
  }
}

template <int W>
inline hipError_t launch_sweep_nr(const SweepArgs& a, hipStream_t stream) {
  if (a.schedule == 2) {
    if constexpr (gl_built(W)) {
      if (a.K >= 1 && a.K <= 64) return launch_sweep_gl<W, 1>(a, stream);
      if (a.K > 64 && a.K <= 128) return launch_sweep_gl<W, 2>(a, stream);
    }
    return hipErrorInvalidValue;
  }
  if (a.schedule == 1) {
    if constexpr (sched_built(W, 1)) return launch_sweep_sc<W, 1>(a, stream);
    return hipErrorInvalidValue;
  }
  return a.schedule == kScheduleLds ? launch_sweep_sc<W, 0>(a, stream) : hipErrorInvalidValue;
}

template <int W, int SC>
inline hipError_t launch_batched_sc(const BatchArgs& a, hipStream_t stream) {
  switch (kc_of(a.K)) {
    case 32: return launch_batched_w<W, 1, 32, SC>(a, stream);
    case 64: return launch_batched_w<W, 1, 64, SC>(a, stream);
    case 112: return launch_batched_w<W, 2, 112, SC>(a, stream);
    case 128: return launch_batched_w<W, 2, 128, SC>(a, stream);
    default: return launch_batched_w<W, 4, 256, SC>(a, stream);
  }
}

template <int W>
inline hipError_t launch_batched_nr(const BatchArgs& a, hipStream_t stream) {
  if (a.schedule == 2) {
    if constexpr (gl_built(W)) {
      if (a.K >= 1 && a.K <= 64) return launch_batched_gl<W, 1>(a, stream);
      if (a.K > 64 && a.K <= 128) return launch_batched_gl<W, 2>(a, stream);
    }
    return hipErrorInvalidValue;
  }
  if (a.schedule == 1) {
    if constexpr (sched_built(W, 1)) return launch_batched_sc<W, 1>(a, stream);
    return hipErrorInvalidValue;
  }
  return a.schedule == kScheduleLds ? launch_batched_sc<W, 0>(a, stream) : hipErrorInvalidValue;
}

template <int W>
inline hipError_t launch_run_nr(const RunArgs& a, hipStream_t stream) {
  switch (kc_of(a.K)) {
    case 32: return launch_run_w<W, 1, 32>(a, stream);
    case 64: return launch_run_w<W, 1, 64>(a, stream);
    case 112: return launch_run_w<W, 2, 112>(a, stream);
    case 128: return launch_run_w<W, 2, 128>(a, stream);
    default: return launch_run_w<W, 4, 256>(a, stream);
  }
}


// Instantiated per code length (words = bits / 64) in tile_mfma_w*.hip.
template <int W>
hipError_t launch_run_words(const RunArgs& a, hipStream_t stream);
template <int W>
hipError_t launch_batched_words(const BatchArgs& a, hipStream_t stream);
template <int W>
hipError_t launch_sweep_words(const SweepArgs& a, hipStream_t stream);

}  // namespace mfma
}  // namespace bdg
