// Matrix-core (MFMA) implicit-GEMM convolutions for the BF16 network.
#include "conv_common.hpp"

namespace mdnp {

void cnn_prepare_mfma_weights(CnnState&, const float*, hipStream_t) {}
bool conv_mfma_supported(int) { return false; }
void conv_mfma_layer(const ConvP&, int, int, int, CnnState&, hipStream_t) {}

}  // namespace mdnp
