// Launch-shape choice of the OMP kernel (omp_kernel.h): lanes per signal and
// correlations per lane.
#include "omp_kernel.h"

namespace dlk {

static int pow2_at_least(int v)
{
    int r = 1;
    while (r < v)
        r <<= 1;
    return r;
}

static int smax_for(int s)
{
    return s <= 4 ? 4 : s <= 6 ? 6 : s <= 8 ? 8 : s <= 12 ? 12 : 16;
}

int omp_smax(int s) { return smax_for(s); }

int omp_signals_per_item(int lps) { return 64 / lps; }

// Default lanes per signal for n atoms at `npl` atoms per lane: enough lanes
// for the atoms and one lane per row of the Cholesky factor.
int omp_lanes_per_signal(int n, int npl, int s)
{
    int lps = pow2_at_least((n + npl - 1) / npl);
    const int need = pow2_at_least(smax_for(s));
    if (lps < need)
        lps = need;
    if (lps < 4)
        lps = 4;
    return lps;
}

// 128 lanes per signal: two waves (with 4 or 8 correlations per lane).
bool omp_config_ok(int n, int s, int lps, int npl)
{
    const bool lps_ok = lps == 4 || lps == 8 || lps == 16 || lps == 32 || lps == 64 ||
                        (lps == 128 && npl <= 8);
    const bool npl_ok = npl == 4 || npl == 8 || npl == 16;
    return lps_ok && npl_ok && lps * npl >= n && lps >= smax_for(s);
}

// 16 correlations per lane, fewer when the group must be wide for L anyway;
// more than 512 atoms with s > 8: two waves per signal of 8 per lane.
int omp_default_npl(int n, int s)
{
    if (n > 512 && smax_for(s) >= 12)
        return 8;  // omp_lanes_per_signal then gives 128
    int npl = 16;
    while (npl > 4 && omp_lanes_per_signal(n, npl, s) * (npl / 2) >= n &&
           omp_lanes_per_signal(n, npl / 2, s) == omp_lanes_per_signal(n, npl, s))
        npl /= 2;
    return npl;
}

hipError_t launch_batched_omp(const OmpArgs *tab, const BatchList &bl, int items, int lps,
                              int npl, int smax, hipStream_t st)
{
    switch (npl) {
    case 4: return launch_omp_batched_npl4(tab, bl, items, lps, smax, st);
    case 8: return launch_omp_batched_npl8(tab, bl, items, lps, smax, st);
    case 16: return launch_omp_batched_npl16(tab, bl, items, lps, smax, st);
    default: return hipErrorInvalidValue;
    }
}

bool omp_carries_error(int n, int s, int lps_req, int npl_req)
{
    const int npl = npl_req > 0 ? npl_req : omp_default_npl(n, s);
    const int lps = lps_req > 0 ? lps_req : omp_lanes_per_signal(n, npl, s);
    return omp_config_ok(n, s, lps, npl) && lps <= 64;
}

hipError_t launch_omp(const OmpArgs &a, hipStream_t st, const RmseArgs *err)
{
    int npl = a.atoms_per_lane;
    if (npl <= 0)
        npl = omp_default_npl(a.n, a.s);
    const int lps = a.lanes_per_signal > 0 ? a.lanes_per_signal
                                           : omp_lanes_per_signal(a.n, npl, a.s);
    if (!omp_config_ok(a.n, a.s, lps, npl) || (err && lps > 64))
        return hipErrorInvalidValue;
    switch (npl) {
    case 4: return launch_omp_npl4(a, lps, st, err);
    case 8: return launch_omp_npl8(a, lps, st, err);
    default: return launch_omp_npl16(a, lps, st, err);
    }
}

}  // namespace dlk
