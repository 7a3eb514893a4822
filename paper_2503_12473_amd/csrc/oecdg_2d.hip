// oecdg_2d.hip -- 2D (tensor Q2) path.  Not yet implemented: every entry
// point reports OECDG_EUNSUPPORTED.
#include "oecdg_internal.h"

namespace oecdg {

int create_2d(oecdg_handle *, const oecdg_desc *) { return OECDG_EUNSUPPORTED; }
int dt_2d(oecdg_handle *, const double *, const double *, double *) { return OECDG_EUNSUPPORTED; }
int stage_2d(oecdg_handle *, int, double, double, const double *, const double *, const double *, const double *,
             double *, double *) {
    return OECDG_EUNSUPPORTED;
}
int run_2d(oecdg_handle *, double *, double *, double, int64_t, double, double *, int64_t *) {
    return OECDG_EUNSUPPORTED;
}
void destroy_2d(oecdg_handle *) {}

}  // namespace oecdg
