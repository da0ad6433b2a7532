// Hamming distance tile on the int8 matrix cores, with the exact top-K fused
// and the neighbour lists carried across column blocks (gfx950 / CDNA4).
//
// The first reduce of the single-pass divide-and-conquer searches every record
// of a partition against all its records exhaustively (Sec. 3.2); the paper
// moved those distance computations to native code (Sec. 3.6 (2)). Here the
// distances are an int8 contraction of a query q as s = 2q - 1 in {-1, +1}^b
// against a candidate a as its {0, 1} bits:
//   <s, a> = popc(q & a) - popc(~q & a) = popc(q) - ham(q, a),
// exact in int32, so ham = popc(q) - dot (on {0,1} vectors the squared
// Euclidean distance of Eq. 1 is the same Hamming distance). Candidates as
// {0, 1} bytes rather than +-1 bytes toggle far fewer bits of the multipliers:
// a throughput probe with random operands sustained 98 % of the int8 peak
// with {0, 1} x +-1 bytes against 88 % with +-1 x +-1.
//
// Operands. A one-off prep kernel writes every code as {0, 1} bytes in the
// operand order of v_mfma_i32_16x16x64_i8: per group of 16 codes and per
// 64-bit word s, a 1 KB fragment whose lane l holds the 16 bytes of code
// (16 g + l % 16), bits [64 s + 16 (l / 16), +16). Loading a fragment is one
// contiguous 16-byte access per lane, into LDS or into registers. The product
// pairs the same code bit of both operands (A and B share the lane-to-k map).
//
// Work split. A work-group has NW compute waves; each owns 16 QG queries
// (rows) held as B operands in registers for the whole job. They share a
// stream of candidate stages (CT codes each) copied from HBM straight into a
// ring of LDS slots (one copy per work-group) and read back as A operands.
// With K <= 64 there are 8 compute waves of 32 queries, two on each SIMD: the
// vector work of one wave (filter, appends, merges, ring bookkeeping) then
// runs while the other's products keep the matrix core busy, which a single
// wave per SIMD cannot do. Longer lists take 4 waves (their LDS leaves no room
// for more). Where registers allow one more wave on a SIMD (codes up to 256
// bits with K <= 64, up to 512 bits with larger K) an extra wave only streams
// the stages and publishes a count of landed ones; otherwise the compute waves
// claim and copy stages themselves.
//
// Filter. The accumulators start at zero, so after the contraction
// acc = popc(q) - ham; adding the per-query bias thr - popc(q) gives thr - ham,
// and a candidate can enter the list only if that is positive. The common case
// (no candidate of a 16-code group beats any of the wave's thresholds) costs a
// max-reduction and one compare per group.
//
// Lists. Keys are dist << IB | column (global column index, IB = 32 - bits
// needed for a distance), so key order is the (distance, index) order of the
// graph. Each job covers one column block [cb, ce): one launch of the run
// kernel, or one work item of the persistent build, which takes a row tile's
// column blocks in order. The lists of its rows are read from the output at
// the start (the merged result of the earlier column blocks, Sec. 3.2 second
// reduce) and written back at the end. Columns arrive in increasing index, so
// an equal distance never displaces a kept key: the strict test ham < thr is
// exact.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "tile_mfma_kern.h"

namespace bdg {
namespace mfma {

// One thread per 16-byte operand chunk; rows >= n are zero (a zero operand
// gives dot 0; such columns are never admitted by the column-range test).
__global__ __launch_bounds__(256) void prep_01_kernel(const uint64_t* __restrict__ codes,
                                                       uint32_t n, uint32_t W, size_t chunks,
                                                       v4i* __restrict__ frags) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= chunks) return;
  const uint32_t l = (uint32_t)(t & 63u);
  const size_t f = t >> 6;  // fragment = group * W + s
  const uint32_t s = (uint32_t)(f % W);
  const size_t row = (f / W) * 16 + (l & 15u);
  v4i v = {0, 0, 0, 0};
  if (row < n) v = code_chunk_01(codes, W, (uint32_t)row, s, l >> 4);
  frags[t] = v;
}

}  // namespace mfma

uint32_t run_idx_bits(uint32_t bits) {
  uint32_t need = 0;
  while ((1u << need) <= bits) ++need;  // distances 0..bits
  return 32u - need;
}

bool run_supported(uint32_t n, uint32_t words, uint32_t K) {
  if (words < 1 || words > 16 || K < 1 || K > 256) return false;
  if ((uint64_t)n > (1ull << run_idx_bits(64 * words)) - 1) return false;
  return mfma::run_lds_bytes(words, K) <= 160 * 1024;
}

bool schedule_supported(uint32_t words, uint32_t K, int schedule) {
  if (schedule == 0 || schedule == kScheduleLds) return true;
  if (schedule == 1) return (words == 2 || words == 4 || words == 8) && K >= 1 && K <= 256;
  if (schedule == 2) return (words == 2 || words == 4 || words == 8) && K >= 1 && K <= 128;
  return false;
}

int resolve_schedule(uint32_t words, uint32_t K, int schedule) {
  if (schedule != 0) return schedule;
  return schedule_supported(words, K, 2) ? 2 : kScheduleLds;
}

size_t prep_rows(uint32_t n) {
  return (((size_t)n + 15) & ~size_t(15)) + 256;  // + at least one stage of slack
}

size_t prep_bytes(uint32_t n, uint32_t words) { return prep_rows(n) * words * 64; }

hipError_t launch_prep(const uint64_t* codes, uint32_t n, uint32_t words, void* frags,
                       hipStream_t stream) {
  const size_t chunks = prep_rows(n) * words * 4;
  dim3 grid((unsigned)((chunks + 255) / 256));
  hipLaunchKernelGGL(mfma::prep_01_kernel, grid, dim3(256), 0, stream, codes, n, words, chunks,
                     reinterpret_cast<mfma::v4i*>(frags));
  return hipGetLastError();
}

uint32_t run_rows_per_wg(uint32_t K) { return (uint32_t)(mfma::nw_of(K) * 16 * mfma::qg_of(K)); }

uint32_t sched_rows_per_wg(uint32_t K, int schedule) {
  return schedule == 2 ? mfma::kGlRows : run_rows_per_wg(K);
}

hipError_t launch_mfma_batched(const BatchArgs& a, hipStream_t stream) {
  if (a.nitems == 0) return hipSuccess;
  switch (a.words) {
    case 1: return mfma::launch_batched_words<1>(a, stream);
    case 2: return mfma::launch_batched_words<2>(a, stream);
    case 3: return mfma::launch_batched_words<3>(a, stream);
    case 4: return mfma::launch_batched_words<4>(a, stream);
    case 5: return mfma::launch_batched_words<5>(a, stream);
    case 6: return mfma::launch_batched_words<6>(a, stream);
    case 7: return mfma::launch_batched_words<7>(a, stream);
    case 8: return mfma::launch_batched_words<8>(a, stream);
    case 9: return mfma::launch_batched_words<9>(a, stream);
    case 10: return mfma::launch_batched_words<10>(a, stream);
    case 11: return mfma::launch_batched_words<11>(a, stream);
    case 12: return mfma::launch_batched_words<12>(a, stream);
    case 13: return mfma::launch_batched_words<13>(a, stream);
    case 14: return mfma::launch_batched_words<14>(a, stream);
    case 15: return mfma::launch_batched_words<15>(a, stream);
    case 16: return mfma::launch_batched_words<16>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

size_t sweep_ctl_words(uint32_t nrows, uint32_t K) {
  const uint32_t rt = run_rows_per_wg(K);
  return 2 + ((size_t)nrows + rt - 1) / rt;
}

hipError_t launch_mfma_sweep(const SweepArgs& a, hipStream_t stream) {
  if (a.nrows == 0 || a.ncols == 0) return hipSuccess;
  if (a.col_block == 0 || a.grid == 0) return hipErrorInvalidValue;
  switch (a.words) {
    case 1: return mfma::launch_sweep_words<1>(a, stream);
    case 2: return mfma::launch_sweep_words<2>(a, stream);
    case 3: return mfma::launch_sweep_words<3>(a, stream);
    case 4: return mfma::launch_sweep_words<4>(a, stream);
    case 5: return mfma::launch_sweep_words<5>(a, stream);
    case 6: return mfma::launch_sweep_words<6>(a, stream);
    case 7: return mfma::launch_sweep_words<7>(a, stream);
    case 8: return mfma::launch_sweep_words<8>(a, stream);
    case 9: return mfma::launch_sweep_words<9>(a, stream);
    case 10: return mfma::launch_sweep_words<10>(a, stream);
    case 11: return mfma::launch_sweep_words<11>(a, stream);
    case 12: return mfma::launch_sweep_words<12>(a, stream);
    case 13: return mfma::launch_sweep_words<13>(a, stream);
    case 14: return mfma::launch_sweep_words<14>(a, stream);
    case 15: return mfma::launch_sweep_words<15>(a, stream);
    case 16: return mfma::launch_sweep_words<16>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mfma_run(const RunArgs& a, hipStream_t stream) {
  if (a.nrows == 0 || a.ce <= a.cb) return hipSuccess;
  switch (a.words) {
    case 1: return mfma::launch_run_words<1>(a, stream);
    case 2: return mfma::launch_run_words<2>(a, stream);
    case 3: return mfma::launch_run_words<3>(a, stream);
    case 4: return mfma::launch_run_words<4>(a, stream);
    case 5: return mfma::launch_run_words<5>(a, stream);
    case 6: return mfma::launch_run_words<6>(a, stream);
    case 7: return mfma::launch_run_words<7>(a, stream);
    case 8: return mfma::launch_run_words<8>(a, stream);
    case 9: return mfma::launch_run_words<9>(a, stream);
    case 10: return mfma::launch_run_words<10>(a, stream);
    case 11: return mfma::launch_run_words<11>(a, stream);
    case 12: return mfma::launch_run_words<12>(a, stream);
    case 13: return mfma::launch_run_words<13>(a, stream);
    case 14: return mfma::launch_run_words<14>(a, stream);
    case 15: return mfma::launch_run_words<15>(a, stream);
    case 16: return mfma::launch_run_words<16>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bdg
