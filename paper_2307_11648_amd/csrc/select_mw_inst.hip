// select_mw_inst.hip -- one (precision, smoothness, waves per column, pool
// rows per lane) family of the multi-wave single-target kernels, compiled
// with CSEL_MW_T (float | double), CSEL_MW_NU (1 | 3 | 5), CSEL_MW_W (2 | 4)
// and CSEL_MW_RPL (1 | 2) defined, so the families build in parallel.
#include "select_mw_kernel.hpp"

#if !defined(CSEL_MW_T) || !defined(CSEL_MW_NU) || !defined(CSEL_MW_W) || !defined(CSEL_MW_RPL)
#error "CSEL_MW_T, CSEL_MW_NU, CSEL_MW_W and CSEL_MW_RPL must be defined"
#endif

#define CSEL_MW_CAT2(a, b, c, d, e) a##_##b##_##c##_##d##_##e
#define CSEL_MW_CAT(a, b, c, d, e) CSEL_MW_CAT2(a, b, c, d, e)

namespace csel {
hipError_t CSEL_MW_CAT(launch_select_mw, CSEL_MW_T, CSEL_MW_NU, CSEL_MW_W, CSEL_MW_RPL)(const SelectArgs& a, int kmax,
                                                                                       hipStream_t s) {
    return launch_mw_impl<CSEL_MW_T, CSEL_MW_NU, CSEL_MW_RPL, CSEL_MW_W>(a, kmax, s);
}
}  // namespace csel
