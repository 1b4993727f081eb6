// Internal interface of the optional per-kernel timing (trace.hip).
#pragma once

#include "common.hpp"

namespace rrf {

enum TraceClass {
  kTrGemm128NN = 0, kTrGemm128TN, kTrGemm128NT, kTrGemm128TT,
  kTrGemm64NN, kTrGemm64TN, kTrGemm64NT, kTrGemm64TT,
  kTrSplitReduce, kTrPanel, kTrJacobi, kTrGaussian, kTrElementwise, kTrGemmBf16,
  kTrGemmGrouped, kTrGemmGrouped128x64, kTrGemmGrouped128x32, kTrGemmGrouped128x16,
  kTrGemmGrouped128x128, kTrGemmX3, kTrGemmX3Small, kTrGemmX6, kTrGemmX6Small, kTrPanelTsqr, kTrCholInv, kTrPanelRecon, kTrPanelFallback, kTraceClasses
};

bool trace_on();
// Returns a token for trace_end (-1 when tracing is off).
int trace_begin(hipStream_t st, int cls, double flops, double bytes);
void trace_end(hipStream_t st, int token);
// Launches on `st` are traced as separate ":UV" classes from now on.
void trace_mark_stream(hipStream_t st);
// ... and as their own classes again.
void trace_unmark_stream(hipStream_t st);
int gemm_trace_class(int tile, bool ta, bool tb);

}  // namespace rrf
