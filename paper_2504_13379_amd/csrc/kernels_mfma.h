// Split-precision W form on the matrix cores (BF16 / FP16 hi + lo).
#pragma once

#include "common.h"
#include "kernels_core.h"

namespace nfr {

constexpr bool kMfmaAvailable = false;

inline bool is_mfma_form(int form) { return form == 2 || form == 3; }
inline size_t mfma_g_bytes(int64_t npad, int B) { return size_t(npad) * B * 8; }
inline int mfma_nsplit(int64_t, int64_t, int) { return 1; }
inline size_t mfma_w_bytes(int64_t n, int64_t npad) { return size_t(n) * npad * 4 + 256; }
inline void launch_mfma_prep(const ProblemView&, int, int, const double*, const Firing&, float*, double*, hipStream_t) {}
inline void launch_mfma_apply(const ProblemView&, int, int, const void*, const float*, double*, hipStream_t) {}
inline void launch_mfma_combine(const ProblemView&, int, int, int, double, double*, double*, double*, const double*, int,
                                const Firing&, float*, hipStream_t) {}
inline void launch_mfma_reduce(const ProblemView&, int, int, const double*, int, double*, hipStream_t) {}
inline void launch_mfma_w_build(const ProblemView&, int, const KernelF64&, void*, hipStream_t) {}

}  // namespace nfr
