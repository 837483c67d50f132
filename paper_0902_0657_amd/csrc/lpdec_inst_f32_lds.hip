// Instantiation of the decode kernels: float PCG vectors, hot arena in LDS.
#include "lpdec_kernels.hpp"

namespace lpdec {
LPDEC_INSTANTIATE(f32_lds, float, true)
}  // namespace lpdec
