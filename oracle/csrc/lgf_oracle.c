/*
 * CPU FP64 oracle: plain lattice-Green's-function direct summation.
 * TEST INFRASTRUCTURE ONLY -- never linked into the product library.
 *
 * Paper, Sec. 2.2, eqs. discrete_laplace / lgf_convolution: the decaying
 * solution of L phi = f on the unbounded lattice is phi = G * f.  With a
 * lattice spacing dx the operator is dx^-2 L, so
 *
 *     u(n) = dx^2 * sum_m G(n - m) f(m)        (no blocking, no FFT)
 *
 * G(n) comes from a dense table of the exact near field, indexed by
 * |n_1|, |n_2|, |n_3| in [0, rn] (the caller builds it from the Bessel
 * integral), and from the asymptotic series beyond max|n_i| > rn
 * (Sec. 5: "asymptotic expansions for far points"; coefficients derived
 * in oracle/derive_far_field.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Asymptotic G(n): -[1/(4 pi r) + Q4/(16 pi r^7) + Q8/(128 pi r^13)
 *                    + Q12/(512 pi r^19)]. */
double oracle_far_field(double x, double y, double z)
{
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double x4 = x2 * x2, y4 = y2 * y2, z4 = z2 * z2;
    const double x6 = x4 * x2, y6 = y4 * y2, z6 = z4 * z2;
    const double x8 = x4 * x4, y8 = y4 * y4, z8 = z4 * z4;
    const double x10 = x8 * x2, y10 = y8 * y2, z10 = z8 * z2;
    const double x12 = x6 * x6, y12 = y6 * y6, z12 = z6 * z6;
    const double r2 = x2 + y2 + z2;
    const double r = sqrt(r2);
    const double q4 = x4 + y4 + z4 - 3.0 * (x2 * y2 + y2 * z2 + z2 * x2);
    const double q8 = 23.0 * (x8 + y8 + z8)
        - 244.0 * (x6 * (y2 + z2) + y6 * (x2 + z2) + z6 * (x2 + y2))
        + 621.0 * (x4 * y4 + y4 * z4 + z4 * x4)
        - 228.0 * x2 * y2 * z2 * r2;
    const double q12 = 647.0 * (x12 + y12 + z12)
        - 16419.0 * (x10 * (y2 + z2) + y10 * (x2 + z2) + z10 * (x2 + y2))
        + 106536.0 * (x8 * (y4 + z4) + y8 * (x4 + z4) + z8 * (x4 + y4))
        - 15723.0 * x2 * y2 * z2 * (x6 + y6 + z6)
        - 178221.0 * (x6 * y6 + y6 * z6 + z6 * x6)
        - 74469.0 * x2 * y2 * z2 * (x4 * (y2 + z2) + y4 * (x2 + z2) + z4 * (x2 + y2))
        + 626835.0 * x4 * y4 * z4;
    const double r7 = r2 * r2 * r2 * r;
    const double r13 = r7 * r2 * r2 * r2;
    const double r19 = r13 * r2 * r2 * r2;
    const double g = 1.0 / (4.0 * M_PI * r) + q4 / (16.0 * M_PI * r7)
                   + q8 / (128.0 * M_PI * r13) + q12 / (512.0 * M_PI * r19);
    return -g;
}

static inline double lookup_G(const double *gnear, int rn, int a, int b, int c)
{
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    c = c < 0 ? -c : c;
    if (a <= rn && b <= rn && c <= rn) {
        const int64_t s = rn + 1;
        return gnear[((int64_t)a * s + b) * s + c];
    }
    return oracle_far_field((double)a, (double)b, (double)c);
}

/* G at a list of lattice points (for table tests). */
void oracle_G_points(const double *gnear, int rn, int64_t n, const int32_t *ijk,
                     double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = lookup_G(gnear, rn, ijk[3 * i], ijk[3 * i + 1], ijk[3 * i + 2]);
}

/*
 * u[t] = scale * sum_s G(tgt[t] - src[s]) * f[s]
 * src_ijk, tgt_ijk: [n][3] integer cell coordinates on one lattice.
 * Each target's sum runs over sources in list order.
 */
void oracle_direct_sum(const double *gnear, int rn,
                       int64_t n_src, const int32_t *src_ijk, const double *f,
                       int64_t n_tgt, const int32_t *tgt_ijk,
                       double scale, double *u)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_tgt; ++t) {
        const int32_t tx = tgt_ijk[3 * t], ty = tgt_ijk[3 * t + 1], tz = tgt_ijk[3 * t + 2];
        double acc = 0.0;
        for (int64_t s = 0; s < n_src; ++s) {
            const double g = lookup_G(gnear, rn, tx - src_ijk[3 * s],
                                      ty - src_ijk[3 * s + 1], tz - src_ijk[3 * s + 2]);
            acc += g * f[s];
        }
        u[t] = scale * acc;
    }
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
