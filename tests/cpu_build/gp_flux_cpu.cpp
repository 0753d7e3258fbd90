// CPU build of the library's Gauss-point flux (csrc/gks_flux_device.h) for
// tests: reads points from stdin, writes the time-integrated fluxes to stdout.
//
// stdin (binary, little endian): int32 n, int32 exact_time, double gamma, mu,
// eps, dt, then per point 48 doubles: WL[4], dL[5][4], WR[4], dR[5][4]
// (face frame; derivative order n, t, nn, nt, tt).  stdout: n x 4 doubles.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../paper_1802_00704_amd/csrc/gks_flux_device.h"

int main() {
    int32_t hdr[2];
    double prm[4];
    if (std::fread(hdr, sizeof(int32_t), 2, stdin) != 2) return 1;
    if (std::fread(prm, sizeof(double), 4, stdin) != 4) return 1;
    const int n = hdr[0];
    gksdev::FluxParams fp;
    fp.gamma = prm[0];
    fp.K = 2.0 / (prm[0] - 1.0) - 2.0;
    fp.mu = prm[1];
    fp.eps = prm[2];
    fp.exact_time = hdr[1];
    const double dt = prm[3];
    std::vector<double> in(48), out(4);
    for (int i = 0; i < n; ++i) {
        if (std::fread(in.data(), sizeof(double), 48, stdin) != 48) return 1;
        double WL[4], dL[5][4], WR[4], dR[5][4];
        for (int q = 0; q < 4; ++q) {
            WL[q] = in[q];
            WR[q] = in[24 + q];
            for (int k = 0; k < 5; ++k) {
                dL[k][q] = in[4 + 4 * k + q];
                dR[k][q] = in[28 + 4 * k + q];
            }
        }
        gksdev::gp_flux(out.data(), WL, dL, WR, dR, dt, fp);
        std::fwrite(out.data(), sizeof(double), 4, stdout);
    }
    return 0;
}
