// Band-inner register-line kernels: float forward instantiations.
#include "kernels_bil.hpp"

namespace fftb {
FFTB_BIL_DECL(, -1, float)
}  // namespace fftb
