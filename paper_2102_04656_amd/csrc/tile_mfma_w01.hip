// Matrix-core tile instantiations for codes of 64..256 bits (words 1..4).
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

template hipError_t launch_run_words<1>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<1>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<1>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<2>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<2>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<2>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<3>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<3>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<3>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<4>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<4>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<4>(const SweepArgs&, hipStream_t);

}  // namespace mfma
}  // namespace bdg
