// Instantiations of the OMP kernel with 4 correlations per lane.
#include "omp_kernel.h"

namespace dlk {

hipError_t launch_omp_npl4(const OmpArgs &a, int lps, hipStream_t st, const RmseArgs *err)
{
    using namespace omp_detail;
    switch (lps) {
    case 4: return launch_omp_s<4, 4>(a, st, err);
    case 8: return launch_omp_s<8, 4>(a, st, err);
    case 16: return launch_omp_s<16, 4>(a, st, err);
    case 32: return launch_omp_s<32, 4>(a, st, err);
    case 64: return launch_omp_s<64, 4>(a, st, err);
    case 128: return launch_omp_pair_s<4>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_omp_batched_npl4(const OmpArgs *tab, const BatchList &bl, int items, int lps,
                                   int smax, hipStream_t st)
{
    using namespace omp_detail;
    switch (lps) {
    case 4: return launch_omp_batched_s<4, 4>(tab, bl, items, smax, st);
    case 8: return launch_omp_batched_s<8, 4>(tab, bl, items, smax, st);
    case 16: return launch_omp_batched_s<16, 4>(tab, bl, items, smax, st);
    case 32: return launch_omp_batched_s<32, 4>(tab, bl, items, smax, st);
    case 64: return launch_omp_batched_s<64, 4>(tab, bl, items, smax, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dlk
