// One launch variant of the fused exchange kernel, chosen at compile time:
// PIMDB_J accumulator rows per thread (1, 2, 4 or 8), PIMDB_BOX (periodic
// minimum image) and PIMDB_MIXED (FP32 compensated pair lengths).  The build
// compiles this file once per variant, in parallel; kernels.hip dispatches
// to the variant a launch needs.
#if !defined(PIMDB_J) || !defined(PIMDB_BOX) || !defined(PIMDB_MIXED)
#error "compile with -DPIMDB_J=<1|2|4|8> -DPIMDB_BOX=<0|1> -DPIMDB_MIXED=<0|1>"
#endif

// this variant's own name for the exponential's coefficient array
#define PIMDB_CAT2(a, b) a##b
#define PIMDB_CAT(a, b) PIMDB_CAT2(a, b)
#define PIMDB_EXP2_SYM PIMDB_CAT(PIMDB_CAT(PIMDB_CAT(exp2_c_j, PIMDB_J), PIMDB_CAT(_b, PIMDB_BOX)), PIMDB_CAT(_m, PIMDB_MIXED))

#include "exchange.h"

namespace pimdb {

template <int J, bool BOX, bool MIXED>
hipError_t launch_exchange_variant(const LaunchArgs &a, int nitems, int threads, int split, hipStream_t st) {
    const size_t smem = exchange_smem_bytes(threads, split == 2);
    if constexpr (J <= 2) {
        if (split) {
            if (threads == 1024 && split == 2)
                hipLaunchKernelGGL((k_exchange_split_wide<J, BOX, MIXED>), dim3(nitems), dim3(threads), smem, st, a);
            else if (threads <= 512)
                hipLaunchKernelGGL((k_exchange_split<J, BOX, MIXED>), dim3(nitems), dim3(threads), smem, st, a);
            else
                return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((k_exchange<J, BOX, MIXED>), dim3(nitems), dim3(threads), smem, st, a);
        }
    } else {
        if (threads > 512 || split) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_exchange_wide<J, BOX, MIXED>), dim3(nitems), dim3(threads), smem, st, a);
    }
    return hipGetLastError();
}

template <int J, bool BOX, bool MIXED>
int exchange_variant_occupancy(int threads, int split) {
    const size_t smem = exchange_smem_bytes(threads, split == 2);
    int n = 0;
    hipError_t e;
    if constexpr (J <= 2) {
        if (split && threads == 1024 && split == 2)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_exchange_split_wide<J, BOX, MIXED>, threads, smem);
        else if (split)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_exchange_split<J, BOX, MIXED>, threads, smem);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_exchange<J, BOX, MIXED>, threads, smem);
    } else {
        if (split) return 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_exchange_wide<J, BOX, MIXED>, threads, smem);
    }
    return e == hipSuccess ? n : 0;
}

template hipError_t launch_exchange_variant<PIMDB_J, (PIMDB_BOX != 0), (PIMDB_MIXED != 0)>(const LaunchArgs &, int, int,
                                                                                       int, hipStream_t);
template int exchange_variant_occupancy<PIMDB_J, (PIMDB_BOX != 0), (PIMDB_MIXED != 0)>(int, int);

} // namespace pimdb
