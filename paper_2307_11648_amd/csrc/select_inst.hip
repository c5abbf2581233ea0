// select_inst.hip -- one (precision, smoothness, gap, pool width) family of
// the single-target kernels.  Compiled once per family with CSEL_SEL_T (float
// | double), CSEL_SEL_NU (1 | 3 | 5), CSEL_SEL_GAP (0 | 1) and CSEL_SEL_RPL
// (1 | 2 | 4 | 8 pool entries per lane) defined, so the fully unrolled
// instantiations build in parallel and each width can take its own
// instruction-scheduling options.
#include "select_kernel.hpp"

#ifndef CSEL_SEL_T
#error "CSEL_SEL_T must be defined"
#endif
#ifndef CSEL_SEL_NU
#error "CSEL_SEL_NU must be defined"
#endif
#ifndef CSEL_SEL_GAP
#error "CSEL_SEL_GAP must be defined"
#endif
#ifndef CSEL_SEL_RPL
#error "CSEL_SEL_RPL must be defined"
#endif

#define CSEL_CAT2(a, b, c, d, e) a##_##b##_##c##_##d##_##e
#define CSEL_CAT(a, b, c, d, e) CSEL_CAT2(a, b, c, d, e)

namespace csel {
hipError_t CSEL_CAT(launch_select, CSEL_SEL_T, CSEL_SEL_NU, CSEL_SEL_GAP, CSEL_SEL_RPL)(const SelectArgs& a, int kmax,
                                                                                      hipStream_t s) {
    return launch_rpl_impl<CSEL_SEL_T, CSEL_SEL_NU, CSEL_SEL_RPL, CSEL_SEL_GAP != 0>(a, kmax, s);
}
}  // namespace csel
