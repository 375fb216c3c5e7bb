/* Driver for the sanitizer build of the oracle's C sources (AddressSanitizer +
 * UBSan, no OpenMP): sweeps and transfer functions on small and odd grids,
 * grids smaller than the velocities, and rejected arguments.  Exit status 0
 * and "OK" on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_sweep(int64_t nx, int64_t ny, int64_t nz, int Q, const int64_t *v, double omega,
                 const double *phi, const double *chi, const double *S, const double *fin,
                 double *fout, double *Phi_out);
int oracle_transfer(int64_t nx, int64_t ny, int64_t nz, int64_t nkx, int Q, const int64_t *v,
                    double omega, const double *phi, const double *chi, double *R);

static double uniform(uint64_t *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0 - 0.5;
}

int main(void)
{
    /* a symmetric 3D set with components up to 3 (27 + 6 velocities) */
    int64_t v[33 * 3];
    int Q = 0;
    for (int a = -1; a <= 1; a++)
        for (int b = -1; b <= 1; b++)
            for (int c = -1; c <= 1; c++) {
                v[3 * Q] = a; v[3 * Q + 1] = b; v[3 * Q + 2] = c; Q++;
            }
    for (int ax = 0; ax < 3; ax++)
        for (int s = -3; s <= 3; s += 6) {
            v[3 * Q] = v[3 * Q + 1] = v[3 * Q + 2] = 0; v[3 * Q + ax] = s; Q++;
        }
    double phi[33], chi[33];
    for (int i = 0; i < Q; i++) { phi[i] = 1.0 / Q; chi[i] = 1.0 / Q; }
    const int64_t grids[][3] = {{1, 1, 1}, {2, 3, 2}, {5, 4, 3}, {7, 1, 1}, {9, 8, 6}};
    uint64_t seed = 42;
    for (unsigned g = 0; g < sizeof grids / sizeof grids[0]; g++) {
        const int64_t nx = grids[g][0], ny = grids[g][1], nz = grids[g][2], n = nx * ny * nz;
        double *S = malloc(sizeof(double) * (size_t)n);
        double *fin = malloc(sizeof(double) * (size_t)(Q * n));
        double *fout = malloc(sizeof(double) * (size_t)(Q * n));
        double *Phi = malloc(sizeof(double) * (size_t)n);
        double *R = malloc(sizeof(double) * (size_t)n);
        for (int64_t c = 0; c < n; c++) S[c] = uniform(&seed);
        for (int64_t c = 0; c < Q * n; c++) fin[c] = uniform(&seed);
        if (oracle_sweep(nx, ny, nz, Q, v, 0.7, phi, chi, S, fin, fout, Phi)) return 1;
        if (oracle_sweep(nx, ny, nz, Q, v, 0.7, phi, chi, S, fout, fin, NULL)) return 1;
        for (int64_t c = 0; c < n; c++)
            if (!isfinite(Phi[c])) return 1;
        if (oracle_transfer(nx, ny, nz, nx, Q, v, 0.8, phi, chi, R)) return 1;
        if (oracle_transfer(nx, ny, nz, nx / 2 + 1, Q, v, 0.8, phi, chi, R)) return 1;
        for (int64_t c = 0; c < n; c++)
            if (!isfinite(R[c])) return 1;
        free(S); free(fin); free(fout); free(Phi); free(R);
    }
    double dummy[8];
    if (oracle_sweep(4, 4, 4, 0, v, 1.0, phi, chi, dummy, dummy, dummy, NULL) == 0) return 1;
    if (oracle_sweep(0, 4, 4, Q, v, 1.0, phi, chi, dummy, dummy, dummy, NULL) == 0) return 1;
    if (oracle_transfer(4, 4, 4, 5, Q, v, 1.0, phi, chi, dummy) == 0) return 1;
    if (oracle_transfer(4, 4, 4, 0, Q, v, 1.0, phi, chi, dummy) == 0) return 1;
    printf("OK\n");
    return 0;
}
