// Instantiations of the OMP kernel with 8 correlations per lane.
#include "omp_kernel.h"

namespace dlk {

hipError_t launch_omp_npl8(const OmpArgs &a, int lps, hipStream_t st, const RmseArgs *err)
{
    using namespace omp_detail;
    switch (lps) {
    case 4: return launch_omp_s<4, 8>(a, st, err);
    case 8: return launch_omp_s<8, 8>(a, st, err);
    case 16: return launch_omp_s<16, 8>(a, st, err);
    case 32: return launch_omp_s<32, 8>(a, st, err);
    case 64: return launch_omp_s<64, 8>(a, st, err);
    case 128: return launch_omp_pair_s<8>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_omp_batched_npl8(const OmpArgs *tab, const BatchList &bl, int items, int lps,
                                   int smax, hipStream_t st)
{
    using namespace omp_detail;
    switch (lps) {
    case 4: return launch_omp_batched_s<4, 8>(tab, bl, items, smax, st);
    case 8: return launch_omp_batched_s<8, 8>(tab, bl, items, smax, st);
    case 16: return launch_omp_batched_s<16, 8>(tab, bl, items, smax, st);
    case 32: return launch_omp_batched_s<32, 8>(tab, bl, items, smax, st);
    case 64: return launch_omp_batched_s<64, 8>(tab, bl, items, smax, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dlk
