// CPU build of the limiter's characteristic basis (csrc/gks_char_basis.h)
// for tests: reads points from stdin, writes L x and R x to stdout.
//
// stdin (binary, little endian): int32 n, double gamma, then per point 10
// doubles: W[4], gx, gy, x[4].  stdout: per point 8 doubles: L x, R x.
#include <cstdint>
#include <cstdio>

#include "../../paper_1802_00704_amd/csrc/gks_char_basis.h"

int main() {
    int32_t n;
    double gamma;
    if (std::fread(&n, sizeof(int32_t), 1, stdin) != 1) return 1;
    if (std::fread(&gamma, sizeof(double), 1, stdin) != 1) return 1;
    for (int i = 0; i < n; ++i) {
        double in[10], out[8];
        if (std::fread(in, sizeof(double), 10, stdin) != 10) return 1;
        gksdev::CharBasis cb;
        cb.init(in, in[4], in[5], gamma);
        cb.to_char(in + 6, out);
        cb.from_char(in + 6, out + 4);
        std::fwrite(out, sizeof(double), 8, stdout);
    }
    return 0;
}
