// Driver of the oracle operation counts: one line of JSON per counted phase,
// operations per DOF (of both meshes).
#include "ora_real.hpp"
#undef double

void count_1d();
void count_2d();

void ora_count_report(const char *name, const ora_count::Counts &c, double per) {
    const double flops = (double)(c.add + c.mul + c.div);
    std::printf("{\"phase\": \"%s\", \"flops_per_dof\": %.3f, \"add\": %.3f, \"mul\": %.3f, \"div\": %.3f, "
                "\"sqrt\": %.3f, \"exp\": %.3f, \"pow\": %.3f, \"minmax_abs\": %.3f, \"compare\": %.3f}\n",
                name, flops / per, c.add / per, c.mul / per, c.div / per, c.sqrt / per, c.exp / per, c.pow / per,
                c.other / per, c.cmp / per);
}

int main() {
    count_1d();
    count_2d();
    return 0;
}
