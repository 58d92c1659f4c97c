// Kernel variants: FP64 gradient.
#include "../../include/gbx.h"
#include "gbx_kernels.h"
#include "gbx_variants.h"

using namespace gbx;

#define V(NN, LL, CC, OO) \
  Variant { GB_FP64, NN, LL, CC, 4, MODE_GRAD, OO, reinterpret_cast<const void*>(&k_batch<double, NN, LL, CC, 4, MODE_GRAD, OO>) }
#define VC(NN, LL, OO) V(NN, LL, 2, OO), V(NN, LL, 3, OO)
// per N: 4 and 8 samples per lane, two register budgets; the first entry is the default
// FP64 gradient: N <= 256 only.  The N = 512 variant faulted once on the GPU (memory aperture
// violation) although a CPU emulation of the same source on the same inputs is clean under
// AddressSanitizer; until the cause is found the FP64 gradient is not offered for N >= 512.
#define VN(OO) VC(64, 16, OO), VC(128, 32, OO), VC(256, 64, OO)

static const Variant kTable[] = {VN(1)};

extern "C" VariantList gbx_variants_f64_grad() { return VariantList{kTable, (int)(sizeof kTable / sizeof kTable[0])}; }
