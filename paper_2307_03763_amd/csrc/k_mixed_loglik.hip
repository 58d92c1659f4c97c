// Kernel variants: mixed-precision log-likelihood.
#include "../../include/gbx.h"
#include "gbx_kernels.h"
#include "gbx_variants.h"

using namespace gbx;

#define V(NN, LL, CC, OO) \
  Variant { GB_MIXED, NN, LL, CC, 4, MODE_LOGLIK, OO, reinterpret_cast<const void*>(&k_batch<float, NN, LL, CC, 4, MODE_LOGLIK, OO>) }
#define VC(NN, LL, OO) V(NN, LL, 2, OO), V(NN, LL, 3, OO)
// per N: 4 and 8 samples per lane, two register budgets; the first entry is the default
#define VN(OO) VC(64, 16, OO), VC(128, 32, OO), VC(256, 64, OO), VC(512, 128, OO), VC(1024, 256, OO), \
               VC(64, 8, OO), VC(128, 16, OO), VC(256, 32, OO), VC(512, 64, OO), VC(1024, 128, OO)

// templates of 128 lanes (two waves) also in workgroups of two waves, one template each, so
// that the template's barriers hold no other template's waves
#define V2(NN, CC, OO) \
  Variant { GB_MIXED, NN, 128, CC, 2, MODE_LOGLIK, OO, reinterpret_cast<const void*>(&k_batch<float, NN, 128, CC, 2, MODE_LOGLIK, OO>) }
#define VW(OO) V2(512, 2, OO), V2(512, 3, OO), V2(1024, 2, OO), V2(1024, 3, OO)

// numerical orbits (one light time per arm): one launch shape per (N, C), not tuned
#define VU(NN, LL, CC) \
  Variant { GB_MIXED, NN, LL, CC, 4, MODE_LOGLIK_UNEQ, 2, reinterpret_cast<const void*>(&k_batch<float, NN, LL, CC, 4, MODE_LOGLIK_UNEQ, 2>) }
#define VUC(NN, LL) VU(NN, LL, 2), VU(NN, LL, 3)

static const Variant kTable[] = {VN(2), VN(4), VW(2), VW(4),
                                 VUC(64, 16), VUC(128, 32), VUC(256, 64), VUC(512, 128), VUC(1024, 256)};

extern "C" VariantList gbx_variants_mixed_loglik() { return VariantList{kTable, (int)(sizeof kTable / sizeof kTable[0])}; }
