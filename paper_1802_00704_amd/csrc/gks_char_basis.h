// Characteristic decomposition of the two-dimensional Euler equations, used
// by the limiter to act on characteristic variables (section 4.2).
//
// Along a unit direction n at a conserved state W = (rho, rho u, rho v, E),
// the Jacobian of F(W).n has eigenvalues u_n - c, u_n, u_n, u_n + c.  The
// columns of R are the matching eigenvectors: the acoustic wave against n,
// the entropy wave, the shear wave and the acoustic wave along n; L = R^-1.
// Both act in closed form on 4-vectors: y = L x and x = R y.
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>

#ifndef GKS_HD
#define GKS_HD __host__ __device__ __forceinline__
#endif

namespace gksdev {

struct CharBasis {
    double u, v, c, ic, H, nx, ny, un, ut, q2, b1, b2;

    // n = (gx, gy) / |(gx, gy)|, the x axis where that vector is zero
    GKS_HD void init(const double W[4], double gx, double gy, double gamma) {
        const double g = hypot(gx, gy);
        nx = g > 0.0 ? gx / g : 1.0;
        ny = g > 0.0 ? gy / g : 0.0;
        const double rho = W[0];
        u = W[1] / rho;
        v = W[2] / rho;
        q2 = u * u + v * v;
        const double p = (gamma - 1.0) * (W[3] - 0.5 * rho * q2);
        c = sqrt(gamma * p / rho);
        ic = 1.0 / c;
        H = (W[3] + p) / rho;
        un = u * nx + v * ny;
        ut = -u * ny + v * nx;
        b1 = (gamma - 1.0) * ic * ic;
        b2 = 0.5 * b1 * q2;
    }
    GKS_HD void to_char(const double x[4], double y[4]) const {
        const double P = b2 * x[0] + b1 * (x[3] - u * x[1] - v * x[2]);
        const double A = ic * (un * x[0] - nx * x[1] - ny * x[2]);
        y[0] = 0.5 * (P + A);
        y[1] = x[0] - P;
        y[2] = -ut * x[0] - ny * x[1] + nx * x[2];
        y[3] = 0.5 * (P - A);
    }
    GKS_HD void from_char(const double y[4], double x[4]) const {
        const double s = y[0] + y[3], d = y[3] - y[0];
        x[0] = s + y[1];
        x[1] = u * x[0] + c * nx * d - ny * y[2];
        x[2] = v * x[0] + c * ny * d + nx * y[2];
        x[3] = H * s + c * un * d + 0.5 * q2 * y[1] + ut * y[2];
    }
};

}  // namespace gksdev
