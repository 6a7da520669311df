// Register-path kernels: F32 inverse, shape part 2.
#include "kernels_reg.hpp"

namespace fftb {
template hipError_t reg_dispatch<+1, float, 2>(int, const KArgs&, int, int, int, int, size_t,
                                              hipStream_t, int, bool, bool*);
}  // namespace fftb
