/*
 * O(N^2) direct sum of the Coulomb potential, the left-hand side of
 * Eq. P2M_phi (no physical constant; the paper writes none), and the field
 * E = -grad(phi).  This is the "exact value" phi_0 of the error measure sigma
 * in Sec. 3.5.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Self-interaction and coincident points are not defined by the paper; the
 * oracle skips j == i and any pair at distance zero.
 */
#include "oracle.h"
#include <math.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int oracle_direct(int64_t n, const double *xyz, const double *q, int64_t nt,
                  const int64_t *targets, double *phi, double *field)
{
    if (n < 0 || nt < 0 || (!targets && nt != n)) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets ? targets[t] : t;
        double s = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = xyz[3 * i] - xyz[3 * j];
            double dy = xyz[3 * i + 1] - xyz[3 * j + 1];
            double dz = xyz[3 * i + 2] - xyz[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            s += q[j] / r;
            double f = q[j] / (r2 * r);
            ex += f * dx; ey += f * dy; ez += f * dz;
        }
        if (phi) phi[t] = s;
        if (field) { field[3 * t] = ex; field[3 * t + 1] = ey; field[3 * t + 2] = ez; }
    }
    return 0;
}
