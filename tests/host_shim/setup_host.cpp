// Host build of the per-cosmology set-up (root finding, root Jacobian) for tests.
#include "../../paper_2212_01937_amd/csrc/setup.hpp"
using namespace cosmo;
extern "C" void host_setup(const double *params, long n, double *out, int *info) {
    for (long c = 0; c < n; ++c) {
        CosmoRec r;
        setup_cosmo(params + 4 * c, r);
        const LaneConst<double> &d = r.d;
        double *o = out + 12 * c;
        o[0] = d.r0; o[1] = 0.0; o[2] = d.r1re; o[3] = d.r1im;
        o[4] = r.pair ? d.r1re : d.r2; o[5] = r.pair ? -d.r1im : 0.0;
        o[6] = d.sigma; o[7] = r.beta; o[8] = r.minsep; o[9] = r.valid; o[10] = r.pair; o[11] = 0.0;
        info[c] = r.info;
    }
}
