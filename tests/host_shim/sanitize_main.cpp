// Stand-alone host driver of the device arithmetic for sanitizer builds (AddressSanitizer,
// UndefinedBehaviorSanitizer): the set-up (roots, root Jacobian, lane constants) and the
// per-lane formulas of both precisions, run over the cosmologies and redshifts of a
// binary input file.  Writes every result to the output file, so that a test can compare
// it with the plain build.
//   input : int64 n_cosmo, int64 n_z, double params[n_cosmo][4], double z[n_z]
//   output: for each cosmology: 12 set-up values and the info word, then per redshift
//           D_C, T, X in FP64 and FP32, the between-redshift D_C and T from z/2 to z and
//           the three time-coordinate Leibniz derivatives (FP64)
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lane_host.cpp"
#include "setup_host.cpp"

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 3;
    long long nc = 0, nz = 0;
    if (fread(&nc, 8, 1, f) != 1 || fread(&nz, 8, 1, f) != 1 || nc <= 0 || nz <= 0) return 4;
    std::vector<double> prm(4 * nc), z(nz);
    if (fread(prm.data(), 8, prm.size(), f) != prm.size() || fread(z.data(), 8, z.size(), f) != z.size()) return 5;
    fclose(f);
    std::vector<double> out;
    std::vector<double> su(12), v(nz), z1(nz), g(3 * nz);
    for (long long i = 0; i < nz; ++i) z1[i] = 0.5 * z[i];
    for (long long c = 0; c < nc; ++c) {
        int info = 0;
        host_setup(prm.data() + 4 * c, 1, su.data(), &info);
        out.insert(out.end(), su.begin(), su.end());
        out.push_back((double)info);
        for (int kind : {COSMO_DC, COSMO_T, COSMO_X})
            for (int dt : {1, 0}) {
                host_eval(prm.data() + 4 * c, kind, dt, z.data(), (long)nz, v.data());
                out.insert(out.end(), v.begin(), v.end());
            }
        for (int kind : {COSMO_DC, COSMO_T}) {
            host_between(prm.data() + 4 * c, kind, 1, z1.data(), z.data(), (long)nz, v.data());
            out.insert(out.end(), v.begin(), v.end());
        }
        host_time_between_grad(prm.data() + 4 * c, 1, z1.data(), z.data(), (long)nz, g.data());
        out.insert(out.end(), g.begin(), g.end());
    }
    FILE *o = fopen(argv[2], "wb");
    if (!o) return 6;
    fwrite(out.data(), 8, out.size(), o);
    fclose(o);
    return 0;
}
