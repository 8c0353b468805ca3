// Host-side helpers shared by the C-ABI sources.
#pragma once

#include <string>

#include "lbw_internal.h"

namespace lbw {

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int validate_desc(const lbw_geometry_desc* d);
// Normalised copy of a descriptor (unused axis 2 of a 2-D grid filled in).
lbw_geometry_desc normalised(const lbw_geometry_desc& d);
// Kernel view of a geometry whose tables live at tab32 / sqrtg.
GeomDev make_geomdev(const lbw_geometry_desc& d, const float* tab32, const double* sqrtg);
// c^2 the kernels step with: the descriptor's c^2 for the corrected
// equilibrium, the effective c_eff^2 = c_s^2 + (c^2 - c_s^2)(1 - D c_s^2) /
// (2 c_s^2), c_s^2 = 1 / (D + 1), for the Hermite form (Sec. II), whose
// collision is the corrected one at that speed on a Cartesian box.
double lattice_c2(const lbw_geometry_desc& d);
int device_cus(int* cus);

}  // namespace lbw

#define HIP_TRY(expr, what)                                          \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) return ::lbw::hip_fail(e_, what);      \
    } while (0)
