// Kernel variants: mixed-precision gradient.
#include "../../include/gbx.h"
#include "gbx_kernels.h"
#include "gbx_variants.h"

using namespace gbx;

#define V(NN, LL, CC, OO) \
  Variant { GB_MIXED, NN, LL, CC, 4, MODE_GRAD, OO, reinterpret_cast<const void*>(&k_batch<float, NN, LL, CC, 4, MODE_GRAD, OO>) }
#define VC(NN, LL, OO) V(NN, LL, 2, OO), V(NN, LL, 3, OO)
// per N: 4 and 8 samples per lane, two register budgets; the first entry is the default
#define VN(OO) VC(64, 16, OO), VC(128, 32, OO), VC(256, 64, OO), VC(512, 128, OO), VC(1024, 256, OO), \
               VC(64, 8, OO), VC(128, 16, OO), VC(256, 32, OO), VC(512, 64, OO), VC(1024, 128, OO)

// templates of 128 lanes (two waves) also in workgroups of two waves, one template each, so
// that the template's barriers hold no other template's waves
#define V2(NN, CC, OO) \
  Variant { GB_MIXED, NN, 128, CC, 2, MODE_GRAD, OO, reinterpret_cast<const void*>(&k_batch<float, NN, 128, CC, 2, MODE_GRAD, OO>) }
#define VW(OO) V2(512, 2, OO), V2(512, 3, OO), V2(1024, 2, OO), V2(1024, 3, OO)

// numerical orbits (one light time per arm): one launch shape per (N, C), not tuned.  The
// register budget of two waves per SIMD: its sample carries three derivative directions and
// needs about 300 registers, so the excess goes to scratch (as in the 3-wave FP64 likelihood
// kernels), not to accumulation registers at one wave per SIMD.
#define VU(NN, LL, CC) \
  Variant { GB_MIXED, NN, LL, CC, 4, MODE_GRAD_UNEQ, 2, reinterpret_cast<const void*>(&k_batch<float, NN, LL, CC, 4, MODE_GRAD_UNEQ, 2>) }
#define VUC(NN, LL) VU(NN, LL, 2), VU(NN, LL, 3)

static const Variant kTable[] = {VN(1), VN(2), VW(1), VW(2),
                                 VUC(64, 16), VUC(128, 32), VUC(256, 64), VUC(512, 128), VUC(1024, 256)};

extern "C" VariantList gbx_variants_mixed_grad() { return VariantList{kTable, (int)(sizeof kTable / sizeof kTable[0])}; }
