/*
 * Plain FP64 sweep of the discrete lattice BGK scheme for the Poisson problem
 * (TEST INFRASTRUCTURE ONLY: the oracle; the product never links this file).
 *
 * One sweep, for every cell x of a periodic nx*ny*nz grid (x fastest):
 *   stream (pull):   f_i(x)   = fin_i(x - v_i)          (indices mod n_axis)
 *   moment:          Phi(x)   = sum_i f_i(x), i = 0..Q-1 in order
 *   collide+source:  fout_i(x) = (1-omega) f_i(x) + omega phi_i Phi(x) + chi_i S(x)
 * which is the BGK relaxation of Eq. (boltzmann) towards the separable
 * equilibrium f_eq = phi(v) Phi (Eq. equilibrium2) with the separable source
 * chi(v) S (Sec. 4), time step 1, omega = 1/tau_lb (Sec. 5).
 * fin/fout hold post-collision populations as Q planes of n cells each.
 * Phi_out (may be NULL) receives the post-stream moment of this sweep.
 * Built with -ffp-contract=off so every product and sum rounds on its own.
 */
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int64_t wrap(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int oracle_sweep(int64_t nx, int64_t ny, int64_t nz, int Q, const int64_t *v,
                 double omega, const double *phi, const double *chi,
                 const double *S, const double *fin, double *fout,
                 double *Phi_out)
{
    const int64_t n = nx * ny * nz;
    if (Q <= 0 || Q > 1024 || n <= 0)
        return 1;
#pragma omp parallel
    {
        double *f = (double *)malloc(sizeof(double) * (size_t)Q);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < n; c++) {
            const int64_t x = c % nx;
            const int64_t y = (c / nx) % ny;
            const int64_t z = c / (nx * ny);
            double Phi = 0.0;
            for (int i = 0; i < Q; i++) {
                const int64_t xs = wrap(x - v[3 * i + 0], nx);
                const int64_t ys = wrap(y - v[3 * i + 1], ny);
                const int64_t zs = wrap(z - v[3 * i + 2], nz);
                f[i] = fin[(int64_t)i * n + (zs * ny + ys) * nx + xs];
                Phi += f[i];
            }
            for (int i = 0; i < Q; i++)
                fout[(int64_t)i * n + c] =
                    (1.0 - omega) * f[i] + omega * phi[i] * Phi + chi[i] * S[c];
            if (Phi_out)
                Phi_out[c] = Phi;
        }
        free(f);
    }
    return 0;
}
