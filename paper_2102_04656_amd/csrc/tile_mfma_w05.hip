// Matrix-core tile instantiations for codes of 320..512 bits (words 5..8).
#include "tile_mfma_kern.h"

namespace bdg {
namespace mfma {

template <int W>
hipError_t launch_run_words(const RunArgs& a, hipStream_t stream) {
  return launch_run_nr<W>(a, stream);
}

template <int W>
hipError_t launch_batched_words(const BatchArgs& a, hipStream_t stream) {
  return launch_batched_nr<W>(a, stream);
}

template <int W>
hipError_t launch_sweep_words(const SweepArgs& a, hipStream_t stream) {
  return launch_sweep_nr<W>(a, stream);
}

template hipError_t launch_run_words<5>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<5>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<5>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<6>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<6>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<6>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<7>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<7>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<7>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<8>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<8>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<8>(const SweepArgs&, hipStream_t);

}  // namespace mfma
}  // namespace bdg
