// Matrix (MFMA) paths: placeholder until the split-precision kernels land.
#include "internal.hpp"

namespace dct {
int mfma_supported(int, int, int) { return 0; }
int mfma_variant_count(int, int, int, int) { return 0; }
int launch_mfma(const DeviceTables*, const Job&, int) { return DCT2D_ERR_PRECISION; }
} // namespace dct
