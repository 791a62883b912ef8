/*
 * gen.c -- seeded synthetic gauge configurations (input generator).
 *
 * This module produces inputs only.  It holds none of the gauge-fixing
 * arithmetic (no functional, no local update, no precision measure), and both
 * the CPU oracle and the GPU library consume its output in the same natural
 * layout: t,x,y,z,mu,i,j,re/im with z fastest, FP64 (18 reals per link).
 *
 * Recipes:
 *   smooth:      U_mu(x) = h(x) exp(i eps sum_a lambda_a xi_{a,mu}(x)) h(x+mu)^dag
 *                with Gell-Mann lambda_a (tr lambda_a lambda_b = 2 delta_ab),
 *                xi ~ N(0,1), h(x) Haar-random SU(3);
 *   pure gauge:  U_mu(x) = h(x) h(x+mu)^dag  (a gauge transform of unit links);
 *   hot:         every link Haar-random;
 *   gauge field: h(x) alone (V x 18 reals), e.g. for random gauge copies.
 * All randoms come from Philox4x64-10 (Salmon et al. 2011) keyed
 * (seed, 0x67656e) with counter (site, slot, block, tag), so every value is a
 * pure function of (seed, site) and independent of thread count or slab.
 * Normals by Box-Muller; Haar matrices by Gram-Schmidt of a complex Gaussian
 * matrix divided by the principal cube root of its determinant (Mezzadri's
 * construction); exp by scaling and squaring of a Taylor series, then a
 * Gram-Schmidt reprojection to SU(3).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cz;

#define GEN_KEY1 0x67656eULL
#define TAG_HAAR 1ULL
#define TAG_XI 2ULL
#define TAG_HOT 3ULL

static void ph_mulhilo(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* Philox4x64 with 10 rounds */
void gen_philox4x64_10(const uint64_t in[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = in[0], x1 = in[1], x2 = in[2], x3 = in[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t h0, l0, h1, l1;
        ph_mulhilo(0xD2E7470EE14C6C93ULL, x0, &h0, &l0);
        ph_mulhilo(0xCA5A826395121157ULL, x2, &h1, &l1);
        uint64_t y0 = h1 ^ x1 ^ k0, y2 = h0 ^ x3 ^ k1;
        x0 = y0;
        x1 = l1;
        x2 = y2;
        x3 = l0;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

static double to_unit(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1.0p-53; }

/* n normals (n even, n <= 24) for (site, slot, tag) */
static void normals(uint64_t seed, uint64_t site, uint64_t slot, uint64_t tag, int n, double *z) {
    const uint64_t key[2] = {seed, GEN_KEY1};
    int made = 0;
    for (uint64_t blk = 0; made < n; ++blk) {
        uint64_t c[4] = {site, slot, blk, tag}, o[4];
        gen_philox4x64_10(c, key, o);
        for (int p = 0; p < 2 && made < n; ++p) {
            double u1 = to_unit(o[2 * p]), u2 = to_unit(o[2 * p + 1]);
            double r = sqrt(-2.0 * log(u1));
            z[made++] = r * cos(2.0 * M_PI * u2);
            z[made++] = r * sin(2.0 * M_PI * u2);
        }
    }
}

typedef struct { cz a[3][3]; } m3;

static m3 m3_mul(const m3 *x, const m3 *y) {
    m3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cz s = 0;
            for (int k = 0; k < 3; ++k) s += x->a[i][k] * y->a[k][j];
            r.a[i][j] = s;
        }
    return r;
}

static m3 m3_mul_dag(const m3 *x, const m3 *y) { /* x y^dag */
    m3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cz s = 0;
            for (int k = 0; k < 3; ++k) s += x->a[i][k] * conj(y->a[j][k]);
            r.a[i][j] = s;
        }
    return r;
}

/* Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): an SU(3) matrix */
static void m3_project(m3 *m) {
    for (int pass = 0; pass < 2; ++pass) {
        double n = 0;
        for (int k = 0; k < 3; ++k) n += creal(m->a[0][k] * conj(m->a[0][k]));
        n = 1.0 / sqrt(n);
        for (int k = 0; k < 3; ++k) m->a[0][k] *= n;
        cz d = 0;
        for (int k = 0; k < 3; ++k) d += conj(m->a[0][k]) * m->a[1][k];
        for (int k = 0; k < 3; ++k) m->a[1][k] -= d * m->a[0][k];
        n = 0;
        for (int k = 0; k < 3; ++k) n += creal(m->a[1][k] * conj(m->a[1][k]));
        n = 1.0 / sqrt(n);
        for (int k = 0; k < 3; ++k) m->a[1][k] *= n;
    }
    m->a[2][0] = conj(m->a[0][1] * m->a[1][2] - m->a[0][2] * m->a[1][1]);
    m->a[2][1] = conj(m->a[0][2] * m->a[1][0] - m->a[0][0] * m->a[1][2]);
    m->a[2][2] = conj(m->a[0][0] * m->a[1][1] - m->a[0][1] * m->a[1][0]);
}

/* Haar-random SU(3) for (seed, site, slot, tag) */
static m3 haar(uint64_t seed, uint64_t site, uint64_t slot, uint64_t tag) {
    double z[18];
    normals(seed, site, slot, tag, 18, z);
    m3 m;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m.a[i][j] = (z[2 * (3 * i + j)] + I * z[2 * (3 * i + j) + 1]) * M_SQRT1_2;
    /* Gram-Schmidt of all three rows gives a Haar unitary */
    for (int r = 0; r < 3; ++r) {
        for (int p = 0; p < r; ++p) {
            cz d = 0;
            for (int k = 0; k < 3; ++k) d += conj(m.a[p][k]) * m.a[r][k];
            for (int k = 0; k < 3; ++k) m.a[r][k] -= d * m.a[p][k];
        }
        double n = 0;
        for (int k = 0; k < 3; ++k) n += creal(m.a[r][k] * conj(m.a[r][k]));
        n = 1.0 / sqrt(n);
        for (int k = 0; k < 3; ++k) m.a[r][k] *= n;
    }
    cz det = m.a[0][0] * (m.a[1][1] * m.a[2][2] - m.a[1][2] * m.a[2][1]) -
             m.a[0][1] * (m.a[1][0] * m.a[2][2] - m.a[1][2] * m.a[2][0]) +
             m.a[0][2] * (m.a[1][0] * m.a[2][1] - m.a[1][1] * m.a[2][0]);
    cz root = cexp(-I * carg(det) / 3.0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m.a[i][j] *= root;
    m3_project(&m);
    return m;
}

/* i * eps * sum_a lambda_a xi_a  (anti-Hermitian, traceless) */
static m3 algebra_element(const double *xi, double eps) {
    const double s3 = 1.0 / sqrt(3.0);
    m3 H;
    memset(&H, 0, sizeof H);
    H.a[0][1] = xi[0] - I * xi[1];
    H.a[1][0] = xi[0] + I * xi[1];
    H.a[0][0] = xi[2] + s3 * xi[7];
    H.a[1][1] = -xi[2] + s3 * xi[7];
    H.a[2][2] = -2.0 * s3 * xi[7];
    H.a[0][2] = xi[3] - I * xi[4];
    H.a[2][0] = xi[3] + I * xi[4];
    H.a[1][2] = xi[5] - I * xi[6];
    H.a[2][1] = xi[5] + I * xi[6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) H.a[i][j] *= I * eps;
    return H;
}

/* exp(X) by scaling and squaring of a degree-14 Taylor series (the scaled
   norm is at most 1/4, so the truncation error is below 1e-17) */
static m3 expm3(const m3 *X) {
    double nrm = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) nrm += cabs(X->a[i][j]);
    int s = 0;
    while (nrm > 0.25 && s < 60) {
        nrm *= 0.5;
        ++s;
    }
    double sc = ldexp(1.0, -s);
    m3 Y;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Y.a[i][j] = X->a[i][j] * sc;
    m3 R, term;
    memset(&R, 0, sizeof R);
    memset(&term, 0, sizeof term);
    for (int i = 0; i < 3; ++i) R.a[i][i] = term.a[i][i] = 1.0;
    for (int k = 1; k <= 14; ++k) {
        term = m3_mul(&term, &Y);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                term.a[i][j] /= (double)k;
                R.a[i][j] += term.a[i][j];
            }
    }
    for (int k = 0; k < s; ++k) R = m3_mul(&R, &R);
    return R;
}

static void put18(double *p, const m3 *m) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            p[2 * (3 * i + j)] = creal(m->a[i][j]);
            p[2 * (3 * i + j) + 1] = cimag(m->a[i][j]);
        }
}

static void coords(const int32_t d[4], int64_t s, int64_t c[4]) {
    for (int k = 3; k >= 0; --k) {
        c[k] = s % d[k];
        s /= d[k];
    }
}

static int64_t fwd_site(const int32_t d[4], int64_t s, int mu) {
    int64_t c[4];
    coords(d, s, c);
    c[mu] = (c[mu] + 1) % d[mu];
    int64_t r = 0;
    for (int k = 0; k < 4; ++k) r = r * d[k] + c[k];
    return r;
}

/* exp(i eps sum lambda_a xi_a) for one link: exported for tests */
void gen_link_exponential(const double xi[8], double eps, double out18[18]) {
    m3 H = algebra_element(xi, eps);
    m3 E = expm3(&H);
    put18(out18, &E);
}

/* the xi_{a,mu}(x) used by gen_smooth for one link */
void gen_link_xi(uint64_t seed, int64_t site, int32_t mu, double xi[8]) {
    normals(seed, (uint64_t)site, (uint64_t)mu, TAG_XI, 8, xi);
}

/* Haar h(x) field on sites [s0, s0+ns): ns x 18 reals */
void gen_haar_field(const int32_t dims[4], uint64_t seed, int64_t s0, int64_t ns, double *out) {
    (void)dims;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ns; ++k) {
        m3 h = haar(seed, (uint64_t)(s0 + k), 4, TAG_HAAR);
        put18(out + 18 * (size_t)k, &h);
    }
}

/* smooth configuration, links of sites with t in [t0, t0+nt): out has
   nt*Nx*Ny*Nz*4*18 reals. eps == 0 with pure != 0 gives the pure gauge.
   h(x) is computed once for the slab and the next time-slice. */
static void smooth_slab(const int32_t dims[4], double eps, uint64_t seed, int32_t t0, int32_t nt, int pure,
                        double *out) {
    const int64_t Vs = (int64_t)dims[1] * dims[2] * dims[3];
    const int64_t s0 = (int64_t)t0 * Vs, ns = (int64_t)nt * Vs;
    m3 *hf = (m3 *)malloc(sizeof(m3) * (size_t)(ns + Vs));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ns + Vs; ++k) {
        int64_t s = s0 + k;
        if (k >= ns) s = ((int64_t)((t0 + nt) % dims[0])) * Vs + (k - ns);
        hf[k] = haar(seed, (uint64_t)s, 4, TAG_HAAR);
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ns; ++k) {
        const int64_t s = s0 + k;
        const m3 *hx = &hf[k];
        for (int mu = 0; mu < 4; ++mu) {
            int64_t y = fwd_site(dims, s, mu);
            /* the forward neighbour in time of the last slice is in the extra slice */
            const int64_t ky = (mu == 0 && s / Vs == (int64_t)t0 + nt - 1) ? ns + (y % Vs) : y - s0;
            const m3 *hy = &hf[ky];
            m3 U;
            if (pure) {
                U = m3_mul_dag(hx, hy);
            } else {
                double xi[8];
                normals(seed, (uint64_t)s, (uint64_t)mu, TAG_XI, 8, xi);
                m3 H = algebra_element(xi, eps);
                m3 E = expm3(&H);
                m3 t = m3_mul(hx, &E);
                U = m3_mul_dag(&t, hy);
            }
            m3_project(&U);
            put18(out + ((size_t)k * 4 + mu) * 18, &U);
        }
    }
    free(hf);
}

void gen_smooth(const int32_t dims[4], double eps, uint64_t seed, int32_t t0, int32_t nt, double *out) {
    smooth_slab(dims, eps, seed, t0, nt, 0, out);
}

void gen_pure_gauge(const int32_t dims[4], uint64_t seed, int32_t t0, int32_t nt, double *out) {
    smooth_slab(dims, 0.0, seed, t0, nt, 1, out);
}

/* every link Haar-random ("hot" start) */
void gen_hot(const int32_t dims[4], uint64_t seed, int32_t t0, int32_t nt, double *out) {
    const int64_t Vs = (int64_t)dims[1] * dims[2] * dims[3];
    const int64_t s0 = (int64_t)t0 * Vs, ns = (int64_t)nt * Vs;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ns; ++k)
        for (int mu = 0; mu < 4; ++mu) {
            m3 h = haar(seed, (uint64_t)(s0 + k), (uint64_t)mu, TAG_HOT);
            put18(out + ((size_t)k * 4 + mu) * 18, &h);
        }
}

/* random gauge copy: U_mu(x) <- h(x) U_mu(x) h(x+mu)^dag with Haar h from
   copy_seed; U holds the whole lattice (natural layout) and is overwritten */
void gen_gauge_copy(const int32_t dims[4], uint64_t copy_seed, double *U) {
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        m3 hx = haar(copy_seed, (uint64_t)s, 4, TAG_HAAR);
        for (int mu = 0; mu < 4; ++mu) {
            m3 hy = haar(copy_seed, (uint64_t)fwd_site(dims, s, mu), 4, TAG_HAAR);
            double *p = U + ((size_t)s * 4 + mu) * 18;
            m3 u;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) u.a[i][j] = p[2 * (3 * i + j)] + I * p[2 * (3 * i + j) + 1];
            m3 t = m3_mul(&hx, &u);
            m3 r = m3_mul_dag(&t, &hy);
            put18(p, &r);
        }
    }
}
