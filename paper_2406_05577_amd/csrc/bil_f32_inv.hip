// Band-inner register-line kernels: float inverse instantiations.
#include "kernels_bil.hpp"

namespace fftb {
FFTB_BIL_DECL(, +1, float)
}  // namespace fftb
