// Registry of compiled kernel variants (one table per translation unit).
#pragma once

namespace gbx {

// k_batch<R, N, LPC, C, WPB, MODE, OCC> (or k_waveform): LPC lanes per template, N / LPC slow-series
// samples per lane, WPB waves per workgroup, OCC the minimum waves per SIMD the register
// allocation must allow (0: no bound).
struct Variant {
  int prec, N, LPC, C, WPB, mode, occ;
  const void* fn;
};

struct VariantList {
  const Variant* v;
  int n;
};

}  // namespace gbx

extern "C" gbx::VariantList gbx_variants_f64_loglik();
extern "C" gbx::VariantList gbx_variants_mixed_loglik();
extern "C" gbx::VariantList gbx_variants_mixed_grad();
extern "C" gbx::VariantList gbx_variants_waveform();
