// Kernel variants: templates on their own bins (gb_waveform).
#include "../../include/gbx.h"
#include "gbx_kernels.h"
#include "gbx_variants.h"

using namespace gbx;

#define W(P, RT, NN, LL, CC) \
  Variant { P, NN, LL, CC, 4, MODE_WAVEFORM, 0, reinterpret_cast<const void*>(&k_waveform<RT, NN, LL, CC, 4>) }
#define WC(P, RT, NN, LL) W(P, RT, NN, LL, 2), W(P, RT, NN, LL, 3)
#define WN(P, RT) WC(P, RT, 64, 16), WC(P, RT, 128, 32), WC(P, RT, 256, 64), WC(P, RT, 512, 128), WC(P, RT, 1024, 256)

// numerical orbits (one light time per arm)
#define WU(P, RT, NN, LL, CC) \
  Variant { P, NN, LL, CC, 4, MODE_WAVEFORM_UNEQ, 0, reinterpret_cast<const void*>(&k_waveform<RT, NN, LL, CC, 4, true>) }
#define WUC(P, RT, NN, LL) WU(P, RT, NN, LL, 2), WU(P, RT, NN, LL, 3)
#define WUN(P, RT) WUC(P, RT, 64, 16), WUC(P, RT, 128, 32), WUC(P, RT, 256, 64), WUC(P, RT, 512, 128), \
                   WUC(P, RT, 1024, 256)

static const Variant kTable[] = {WN(GB_FP64, double), WN(GB_MIXED, float), WUN(GB_FP64, double), WUN(GB_MIXED, float)};

extern "C" VariantList gbx_variants_waveform() { return VariantList{kTable, (int)(sizeof kTable / sizeof kTable[0])}; }
