// One launch variant of the fused exchange kernel, chosen at compile time:
// PIMDB_J accumulator rows per thread (1, 2, 4 or 8), PIMDB_BOX (periodic
// minimum image) and PIMDB_MIXED (FP32 compensated pair lengths).  The build
// compiles this file once per variant, in parallel; kernels.hip dispatches
// to the variant a launch needs.
#include "exchange.h"

#if !defined(PIMDB_J) || !defined(PIMDB_BOX) || !defined(PIMDB_MIXED)
#error "compile with -DPIMDB_J=<1|2|4|8> -DPIMDB_BOX=<0|1> -DPIMDB_MIXED=<0|1>"
#endif

namespace pimdb {

template <int J, bool BOX, bool MIXED>
hipError_t launch_exchange_variant(const LaunchArgs &a, int nitems, int threads, hipStream_t st) {
    const size_t smem = exchange_smem_bytes(threads);
    if constexpr (J <= 2) {
        hipLaunchKernelGGL((k_exchange<J, BOX, MIXED>), dim3(nitems), dim3(threads), smem, st, a);
    } else {
        if (threads > 512) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_exchange_wide<J, BOX, MIXED>), dim3(nitems), dim3(threads), smem, st, a);
    }
    return hipGetLastError();
}

template hipError_t launch_exchange_variant<PIMDB_J, (PIMDB_BOX != 0), (PIMDB_MIXED != 0)>(const LaunchArgs &, int, int,
                                                                                       hipStream_t);

} // namespace pimdb
