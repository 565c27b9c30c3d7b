// Launches of the vector-ALU filter with the channel-Fourier threshold
// (RGB; kernel template in filter_valu.h), in a translation unit of their
// own so that they compile in parallel with the other variants.
#include "filter_valu.h"

namespace hts {

template <int MASKS, int BATCH, int WT>
static hipError_t launch_ft(const Launch& L, int g, size_t lds, hipStream_t s) {
  switch (L.K) {
    case 2: case 4: case 8:
      hipLaunchKernelGGL((k_filter<3, 1, 0, MASKS, BATCH, WT, 1>), dim3(g), dim3(256), lds, s, L); break;
    case 16:
      hipLaunchKernelGGL((k_filter<3, 2, 0, MASKS, BATCH, WT, 1>), dim3(g), dim3(256), lds, s, L); break;
    case 32:
      hipLaunchKernelGGL((k_filter<3, 4, 0, MASKS, BATCH, WT, 1>), dim3(g), dim3(256), lds, s, L); break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_filter_ft(const Launch& L, int g, size_t lds, bool batch, bool masks, bool wt,
                            hipStream_t s) {
  if (wt) {
    if (batch) return launch_ft<0, 1, 1>(L, g, lds, s);
    return masks ? launch_ft<1, 0, 1>(L, g, lds, s) : launch_ft<0, 0, 1>(L, g, lds, s);
  }
  if (batch) return launch_ft<0, 1, 0>(L, g, lds, s);
  return masks ? launch_ft<1, 0, 0>(L, g, lds, s) : launch_ft<0, 0, 0>(L, g, lds, s);
}

}  // namespace hts
