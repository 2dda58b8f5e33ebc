/* Precision floor of the Heston Euler sweep (full truncation, log-price x,
 * variance v) at a parameter point: E y_i over P paths computed twice on the
 * same normals, once in FP64 and once with every normal and every result of
 * the variance recursion (v+, sqrt(v+), w, v) rounded to k significant bits
 * (k = 24 is the rounding of FP32 storage; the log-price stays FP64 so that
 * only the variance recursion's precision is varied).  Prints the largest
 * relative price error max_i |dEy_i| / max(|Ey_i|, 1e-2).
 *
 * Test-only program: its own Philox4x32-10 (Salmon et al. 2011) and
 * Box-Muller, sharing no code with the library or the oracle.  Instruments:
 * 8 strikes 70..130 x 5 maturities at steps 32, 88, 144, 200, 256 of
 * N = 256 steps over 2 years; S0 = 100, r = 0.02; Philox key 1, counter
 * (call, path, 0, 0).
 *
 * usage: precision_floor P k kappa theta_bar xi rho v0 [kz]   (kz defaults to k) */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

static void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, uint32_t o[4])
{
    for (int r = 0; r < 10; ++r) {
        uint64_t a = (uint64_t)0xD2511F53u * c0, b = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0, n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o[0] = c0; o[1] = c1; o[2] = c2; o[3] = c3;
}

/* v rounded to k significant bits (round to nearest) */
static double rnd(double v, int k)
{
    if (v == 0.0 || k >= 53) return v;
    int e;
    double f = frexp(v, &e);
    double s = ldexp(1.0, k);
    return ldexp(nearbyint(f * s) / s, e);
}

#define NSTEP 256
#define NINS 40

int main(int argc, char **argv)
{
    if (argc != 8 && argc != 9) return 2;
    const long P = atol(argv[1]);
    const int k = atoi(argv[2]);
    const int kz = argc == 9 ? atoi(argv[8]) : k;
    const double kap = atof(argv[3]), thb = atof(argv[4]), xi = atof(argv[5]), rho = atof(argv[6]),
                 v0 = atof(argv[7]);
    const double h = 2.0 / NSTEP, sq = sqrt(h), r = 0.02, s0 = 100.0, rhop = sqrt(1.0 - rho * rho);
    const int date[5] = {32, 88, 144, 200, 256};
    double sum_a[NINS] = {0}, sum_b[NINS] = {0};
#pragma omp parallel for reduction(+ : sum_a[:NINS], sum_b[:NINS]) schedule(static)
    for (long p = 0; p < P; ++p) {
        double xa = 0, va = v0, xb = 0, vb = v0;
        int d = 0;
        for (int call = 0; call < NSTEP / 2; ++call) {
            uint32_t w[4];
            philox((uint32_t)call, (uint32_t)p, 0u, 0u, 1u, 0u, w);
            for (int j = 0; j < 2; ++j) {
                const double u0 = ((double)(w[2 * j] >> 9) + 0.5) * 0x1p-23;
                const double u1 = ((double)(w[2 * j + 1] >> 9) + 0.5) * 0x1p-23;
                const double rr = sqrt(-2.0 * log(u0));
                const double z1 = rr * cos(2.0 * M_PI * u1), z2 = rr * sin(2.0 * M_PI * u1);
                /* FP64 sweep */
                double vp = va > 0 ? va : 0, s = sqrt(vp);
                double xn = xa + (r - 0.5 * vp) * h + s * sq * z1;
                va = va + kap * (thb - vp) * h + xi * s * sq * (rho * z1 + rhop * z2);
                xa = xn;
                /* the same with k-bit normals and variance recursion */
                const double y1 = rnd(z1, kz), y2 = rnd(z2, kz);
                vp = rnd(vb > 0 ? vb : 0, k);
                s = rnd(sqrt(vp), k);
                const double ww = rnd(rho * y1 + rhop * y2, k);
                xb = xb + (r - 0.5 * vp) * h + s * sq * y1;
                vb = rnd(vb + kap * (thb - vp) * h + xi * s * sq * ww, k);
                const int n = 2 * call + j + 1;
                if (n == date[d]) {
                    const double disc = exp(-r * n * h), Sa = s0 * exp(xa), Sb = s0 * exp(xb);
                    for (int i = 0; i < 8; ++i) {
                        const double K = 70.0 + 60.0 * i / 7.0;
                        sum_a[8 * d + i] += disc * fmax(Sa - K, 0.0);
                        sum_b[8 * d + i] += disc * fmax(Sb - K, 0.0);
                    }
                    ++d;
                }
            }
        }
    }
    double worst = 0.0;
    for (int i = 0; i < NINS; ++i) {
        const double e = fabs(sum_b[i] - sum_a[i]) / P / fmax(fabs(sum_a[i]) / P, 1e-2);
        if (e > worst) worst = e;
    }
    printf("%.6e\n", worst);
    return 0;
}
