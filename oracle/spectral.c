/*
 * Transfer function of the exact fixed point on a periodic grid, in plain C
 * (TEST INFRASTRUCTURE ONLY: the oracle; the product never links this file).
 *
 * The sweep is linear and shift-invariant, so each Fourier mode k settles on
 * its own.  For a lattice closed under v -> -v with even phi, chi and
 * a = 1 - omega, theta_i = k.v_i, s_i = sin(theta_i / 2):
 *   D(k) = sum_i phi_i 2 (2 - omega) s_i^2 / (omega^2 + 4 a s_i^2)
 *   A(k) = sum_i chi_i (cos theta_i - a) / (omega^2 + 4 a s_i^2)
 *   Phi_hat(k) = S_hat(k) A(k) / D(k),   Phi_hat(0) = 0.
 * This is the formula of oracle/spectral.py (``transfer``), evaluated here for
 * large grids: the phase k.v_i = 2 pi p / L with L = lcm(nx, ny, nz) and the
 * integer p reduced exactly to (-L/2, L/2], so sin and cos come from two
 * tables of L entries built once.
 *
 * Modes: mx in [0, nkx), my in [0, ny), mz in [0, nz); R is stored
 * R[(mz * ny + my) * nkx + mx].  nkx = nx gives every mode, nkx = nx/2 + 1
 * the half spectrum of a real FFT (R is even in k).
 * Built with -ffp-contract=off so every product and sum rounds on its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static int64_t gcd64(int64_t a, int64_t b)
{
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

static int64_t lcm64(int64_t a, int64_t b) { return a / gcd64(a, b) * b; }

int oracle_transfer(int64_t nx, int64_t ny, int64_t nz, int64_t nkx, int Q, const int64_t *v,
                    double omega, const double *phi, const double *chi, double *R)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || nkx <= 0 || nkx > nx || Q <= 0 || Q > 1024)
        return 1;
    const int64_t L = lcm64(lcm64(nx, ny), nz);
    if (L > ((int64_t)1 << 28))
        return 2;
    const double pi = 3.14159265358979323846;
    const double a = 1.0 - omega;
    double *s2t = (double *)malloc(sizeof(double) * (size_t)L);
    double *ct = (double *)malloc(sizeof(double) * (size_t)L);
    if (!s2t || !ct) {
        free(s2t);
        free(ct);
        return 3;
    }
    for (int64_t p = 0; p < L; p++) {
        const int64_t q = p > L / 2 ? p - L : p; /* theta in (-pi, pi] */
        const double theta = (2.0 * pi / (double)L) * (double)q;
        const double s = sin(0.5 * theta);
        s2t[p] = s * s;
        ct[p] = cos(theta);
    }
    const int64_t fx = L / nx, fy = L / ny, fz = L / nz;
#pragma omp parallel for schedule(static)
    for (int64_t row = 0; row < nz * ny; row++) {
        const int64_t mz = row / ny, my = row % ny;
        for (int64_t mx = 0; mx < nkx; mx++) {
            double A = 0.0, D = 0.0;
            for (int i = 0; i < Q; i++) {
                int64_t p = (mx * v[3 * i + 0] * fx + my * v[3 * i + 1] * fy + mz * v[3 * i + 2] * fz) % L;
                if (p < 0)
                    p += L;
                const double s2 = s2t[p];
                const double den = omega * omega + 4.0 * a * s2;
                A = A + chi[i] * (ct[p] - a) / den;
                D = D + phi[i] * 2.0 * (2.0 - omega) * s2 / den;
            }
            R[row * nkx + mx] = (D != 0.0 && (mx | my | mz) != 0) ? A / D : 0.0;
        }
    }
    free(s2t);
    free(ct);
    return 0;
}
