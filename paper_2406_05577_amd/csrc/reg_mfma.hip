// Register-path kernels with the FP32 DFT_16 on the matrix cores.
#include "kernels_reg.hpp"

namespace fftb {
template hipError_t reg_dispatch_mfma<+1>(int, const KArgs&, int, int, size_t, hipStream_t, int, bool);
template hipError_t reg_dispatch_mfma<-1>(int, const KArgs&, int, int, size_t, hipStream_t, int, bool);
}  // namespace fftb
