// Matrix-core tile instantiations for codes of 576..768 bits (words 9..12).
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

template hipError_t launch_run_words<9>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<9>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<9>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<10>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<10>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<10>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<11>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<11>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<11>(const SweepArgs&, hipStream_t);
template hipError_t launch_run_words<12>(const RunArgs&, hipStream_t);
template hipError_t launch_batched_words<12>(const BatchArgs&, hipStream_t);
template hipError_t launch_sweep_words<12>(const SweepArgs&, hipStream_t);

}  // namespace mfma
}  // namespace bdg
