// select_inst.hip -- one (precision, smoothness, gap) family of the
// single-target kernels.  Compiled once per family with CSEL_SEL_T (float |
// double), CSEL_SEL_NU (1 | 3 | 5) and CSEL_SEL_GAP (0 | 1) defined, so the
// fully unrolled instantiations build in parallel.
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

#define CSEL_CAT2(a, b, c, d) a##_##b##_##c##_##d
#define CSEL_CAT(a, b, c, d) CSEL_CAT2(a, b, c, d)

namespace csel {
hipError_t CSEL_CAT(launch_select, CSEL_SEL_T, CSEL_SEL_NU, CSEL_SEL_GAP)(const SelectArgs& a, int rpl, int kmax,
                                                                         hipStream_t s) {
    return launch_nu_impl<CSEL_SEL_T, CSEL_SEL_NU, CSEL_SEL_GAP != 0>(a, rpl, kmax, s);
}
}  // namespace csel
