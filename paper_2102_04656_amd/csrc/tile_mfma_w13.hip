// Matrix-core tile instantiations for codes of 832..1024 bits (words 13..16).
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

template hipError_t launch_run_words<13>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<13>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<13>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<14>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<14>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<14>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<15>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<15>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<15>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<16>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<16>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<16>(const SweepArgs&, hipStream_t);

}  // namespace mfma
}  // namespace bdg
