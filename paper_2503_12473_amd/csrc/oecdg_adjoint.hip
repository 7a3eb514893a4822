// oecdg_adjoint.hip -- discrete adjoint of the 1D RK-OECDG run.  Not yet
// implemented: reports OECDG_EUNSUPPORTED.
#include "oecdg_internal.h"

namespace oecdg {

int adjoint_1d(oecdg_handle *, const double *, const double *, int64_t, double, const double *, const double *,
               double *, double *, int) {
    return OECDG_EUNSUPPORTED;
}

}  // namespace oecdg
