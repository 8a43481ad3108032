// Z_{2^64} matrix products on int8 MFMA (8-bit balanced limbs), gfx950.
#include "gemm.h"

namespace mpc3 {

hipError_t gemm_u64(const GemmArgs& g, hipStream_t stream);

hipError_t gemm_limb(const GemmArgs& g, hipStream_t stream) { return gemm_u64(g, stream); }

}  // namespace mpc3
