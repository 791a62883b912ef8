/*
 * gf_oracle.c -- plain FP64 CPU oracle for SU(3) and SU(2) lattice gauge fixing
 * (Schroeck & Vogt, "Coulomb, Landau and Maximally Abelian Gauge Fixing in
 * Lattice QCD with Multi-GPUs", arXiv:1212.5221).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference the GPU path is checked against.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no code
 * with the HIP library: no header, no helper, no table.
 *
 * Everything is double precision, written to be read against the paper:
 *   - links in the natural ("StandardPattern", Sec. 4.2.1) order
 *     t,x,y,z,mu,i,j,re/im with z fastest; periodic boundaries;
 *   - Alg. 1 (Sec. 2.4): for parity even then odd, for every site of that
 *     parity, for every SU(2) subgroup (0,1),(0,2),(1,2): Step 1 computes the
 *     local g(x) from the *current* adjacent links, Step 2 applies it to the
 *     eight (Coulomb: six) adjacent links before the next subgroup;
 *   - no algebraic shortcut, no fusion: K(x) is rebuilt from the links for
 *     every subgroup.
 *
 * Readings where the paper is silent or inconsistent (each also listed in the
 * design notes of the repository):
 *   R1 periodic boundary conditions, even extents;
 *   R2 subgroup order (0,1),(0,2),(1,2);
 *   R3 Landau/Coulomb local optimum of Re tr[gK] is the conjugate of the
 *      subgroup quaternion of K, normalised (Sec. 2.2.1, eq. localsolution);
 *   R4 MAG: the coefficient D of the quadratic form (Sec. 2.2.2, eq. upMatrix)
 *      must be twice the printed value to agree with eq. (up); the SU(3) block
 *      form below reduces to that for SU(2) links;
 *   R5 overrelaxation is the printed first-order map (App. A, Fig.
 *      calculateUpdate) applied to the normalised relaxation quaternion;
 *   R6 microcanonical step = exact square of the relaxation quaternion
 *      (Sec. 2.2.4 claims invariance of the local functional; only the exact
 *      square has it);
 *   R7 A_mu = traceless part of (U - U^dag)/(2i), from U = exp(i a g A)
 *      (Sec. 1), fixing the scale of theta (Sec. 2.1.1);
 *   R8 MAG theta (Sec. 2.1.2) for SU(3): sum over i<j of |Gamma_ij|^2 with
 *      Gamma = W - W^dag, W = sum_mu [U D(U)^dag - D(U')^dag U'], D() the
 *      diagonal part, U' the backward link; the literal squared-sum form is
 *      reported separately (gfo_theta_mag_literal: parity unpinned, the
 *      printed form being ambiguous; nothing depends on it);
 *   R9 Coulomb: 3D parity (x+y+z) mod 2 inside each time-slice, F and theta
 *      normalised per time-slice with 3 spatial directions, G(x) accumulates
 *      the transformation, U_0(x) <- G(x) U_0(x) G(x+0)^dag at the end
 *      (Sec. 5, the final g(t) applied to U_0(t-1));
 *   R10 heatbath (Sec. 2.3): Landau/Coulomb g = r.h with r_0 drawn from
 *      sqrt(1-r0^2) exp(a r0) (Creutz for a<2, Kennedy-Pendleton else, 64
 *      tries then r=1); MAG exact von Mises-Fisher on S^2 for n(g); randoms
 *      from Philox4x64-10 keyed (seed, instance), counter (sweep, site,
 *      subgroup<<16 | block, stream);
 *   R11 annealing schedule linear in T, one heatbath sweep then nmicro
 *      microcanonical sweeps per step;
 *   R12 SU(2) gauge group (functions gfo2_*): the MAG term of the backward
 *      link U_mu(x - mu), which transforms as U_mu(x - mu) g(x)^dag, is the
 *      forward term of U_mu(x - mu)^dag (the printed local functional leaves
 *      the second term to the reader); the heatbath weight is
 *      exp(Re tr[g K] / T) as for an SU(3) subgroup;
 *   R13 reprojection inside a run (Sec. 4.5; the interval is the caller's):
 *      after every reunit_every sweeps the links of every unit still running
 *      are reprojected, and for Coulomb gauge the accumulated G(x) of those
 *      time-slices too; a time-slice that has stopped keeps exactly the links
 *      its stopping check measured (its links are neither updated nor
 *      reprojected any more).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { GFO_LANDAU = 0, GFO_COULOMB = 1, GFO_MAG = 2 };
enum { GFO_OR = 0, GFO_MICRO = 1, GFO_HEATBATH = 2, GFO_SR = 3 };

/* ------------------------------------------------------------------ */
/* Geometry (Sec. 4.2.1 StandardPattern; Sec. 2.4 parity footnote)     */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n[4]; /* n[0]=Nt, n[1]=Nx, n[2]=Ny, n[3]=Nz */
    int64_t V;
} geom;

static geom make_geom(const int32_t dims[4]) {
    geom g;
    g.V = 1;
    for (int d = 0; d < 4; ++d) {
        g.n[d] = dims[d];
        g.V *= dims[d];
    }
    return g;
}

static void site_coords(const geom *g, int64_t s, int64_t c[4]) {
    for (int d = 3; d >= 0; --d) {
        c[d] = s % g->n[d];
        s /= g->n[d];
    }
}

static int64_t coords_site(const geom *g, const int64_t c[4]) {
    int64_t s = 0;
    for (int d = 0; d < 4; ++d) s = s * g->n[d] + c[d];
    return s;
}

/* neighbour x + dir*mu_hat, periodic */
static int64_t site_shift(const geom *g, int64_t s, int mu, int dir) {
    int64_t c[4];
    site_coords(g, s, c);
    c[mu] = (c[mu] + dir + g->n[mu]) % g->n[mu];
    return coords_site(g, c);
}

static int site_parity4(const geom *g, int64_t s) {
    int64_t c[4];
    site_coords(g, s, c);
    return (int)((c[0] + c[1] + c[2] + c[3]) & 1);
}

static int site_parity3(const geom *g, int64_t s) {
    int64_t c[4];
    site_coords(g, s, c);
    return (int)((c[1] + c[2] + c[3]) & 1);
}

static int64_t site_t(const geom *g, int64_t s) {
    int64_t c[4];
    site_coords(g, s, c);
    return c[0];
}

/* ------------------------------------------------------------------ */
/* SU(3) matrices in the natural layout                                */
/* ------------------------------------------------------------------ */

typedef struct { cplx e[3][3]; } mat3;

static mat3 link_get(const double *U, int64_t s, int mu) {
    mat3 m;
    const double *p = U + ((size_t)s * 4 + (size_t)mu) * 18;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m.e[i][j] = CMPLX(p[(i * 3 + j) * 2], p[(i * 3 + j) * 2 + 1]);
    return m;
}

static void link_put(double *U, int64_t s, int mu, const mat3 *m) {
    double *p = U + ((size_t)s * 4 + (size_t)mu) * 18;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            p[(i * 3 + j) * 2] = creal(m->e[i][j]);
            p[(i * 3 + j) * 2 + 1] = cimag(m->e[i][j]);
        }
}

static mat3 mat_get18(const double *p) {
    mat3 m;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m.e[i][j] = CMPLX(p[(i * 3 + j) * 2], p[(i * 3 + j) * 2 + 1]);
    return m;
}

static void mat_put18(double *p, const mat3 *m) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            p[(i * 3 + j) * 2] = creal(m->e[i][j]);
            p[(i * 3 + j) * 2 + 1] = cimag(m->e[i][j]);
        }
}

static mat3 mat_identity(void) {
    mat3 m;
    memset(&m, 0, sizeof m);
    for (int i = 0; i < 3; ++i) m.e[i][i] = 1.0;
    return m;
}

static mat3 mat_zero(void) {
    mat3 m;
    memset(&m, 0, sizeof m);
    return m;
}

static mat3 mat_dag(const mat3 *a) {
    mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.e[i][j] = conj(a->e[j][i]);
    return r;
}

static mat3 mat_mul(const mat3 *a, const mat3 *b) {
    mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a->e[i][k] * b->e[k][j];
            r.e[i][j] = s;
        }
    return r;
}

static void mat_acc(mat3 *a, const mat3 *b) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a->e[i][j] += b->e[i][j];
}

static double mat_retrace(const mat3 *a) { return creal(a->e[0][0] + a->e[1][1] + a->e[2][2]); }

static cplx mat_det(const mat3 *a) {
    return a->e[0][0] * (a->e[1][1] * a->e[2][2] - a->e[1][2] * a->e[2][1]) -
           a->e[0][1] * (a->e[1][0] * a->e[2][2] - a->e[1][2] * a->e[2][0]) +
           a->e[0][2] * (a->e[1][0] * a->e[2][1] - a->e[1][1] * a->e[2][0]);
}

/* traceless part of (M - M^dag)/(2i)  (reading R7) */
static mat3 mat_antiherm_traceless(const mat3 *m) {
    mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.e[i][j] = (m->e[i][j] - conj(m->e[j][i])) / (2.0 * I);
    cplx tr = (r.e[0][0] + r.e[1][1] + r.e[2][2]) / 3.0;
    for (int i = 0; i < 3; ++i) r.e[i][i] -= tr;
    return r;
}

/* tr(A A^dag) = sum |A_ij|^2 */
static double mat_norm2(const mat3 *a) {
    double s = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s += creal(a->e[i][j]) * creal(a->e[i][j]) + cimag(a->e[i][j]) * cimag(a->e[i][j]);
    return s;
}

/* Reprojection to SU(3) (Sec. 4.5): normalise row 0, Gram-Schmidt row 1,
   row 2 = (row0 x row1)^*  (Sec. 4.2, third row from the first two). */
static void mat_reunitarise(mat3 *m) {
    double n0 = 0;
    for (int k = 0; k < 3; ++k) n0 += creal(m->e[0][k] * conj(m->e[0][k]));
    n0 = 1.0 / sqrt(n0);
    for (int k = 0; k < 3; ++k) m->e[0][k] *= n0;
    cplx p = 0;
    for (int k = 0; k < 3; ++k) p += conj(m->e[0][k]) * m->e[1][k];
    for (int k = 0; k < 3; ++k) m->e[1][k] -= p * m->e[0][k];
    double n1 = 0;
    for (int k = 0; k < 3; ++k) n1 += creal(m->e[1][k] * conj(m->e[1][k]));
    n1 = 1.0 / sqrt(n1);
    for (int k = 0; k < 3; ++k) m->e[1][k] *= n1;
    const cplx *u = m->e[0], *v = m->e[1];
    m->e[2][0] = conj(u[1] * v[2] - u[2] * v[1]);
    m->e[2][1] = conj(u[2] * v[0] - u[0] * v[2]);
    m->e[2][2] = conj(u[0] * v[1] - u[1] * v[0]);
}

/* ------------------------------------------------------------------ */
/* SU(2) subgroup elements as quaternions (Sec. 2.2.2, Cayley-Klein)   */
/*   g = [[g0 + i g3,  g2 + i g1], [-g2 + i g1,  g0 - i g3]]           */
/* ------------------------------------------------------------------ */

typedef struct { double v[4]; } quat;

static void quat_to_2x2(quat g, cplx m[2][2]) {
    m[0][0] = CMPLX(g.v[0], g.v[3]);
    m[0][1] = CMPLX(g.v[2], g.v[1]);
    m[1][0] = CMPLX(-g.v[2], g.v[1]);
    m[1][1] = CMPLX(g.v[0], -g.v[3]);
}

/* App. A, Fig. getSubgroupQuaternion: the 2x2 block (i,j) of M as 4 reals */
static quat subgroup_quaternion(const mat3 *M, int i, int j) {
    quat q;
    q.v[0] = creal(M->e[i][i]) + creal(M->e[j][j]);
    q.v[3] = cimag(M->e[i][i]) - cimag(M->e[j][j]);
    q.v[2] = creal(M->e[i][j]) - creal(M->e[j][i]);
    q.v[1] = cimag(M->e[i][j]) + cimag(M->e[j][i]);
    return q;
}

/* App. A, Fig. subgroupmult: rows i,j of M <- g (2x2) times rows i,j */
static void left_subgroup_mult(mat3 *M, int i, int j, quat g) {
    cplx h[2][2];
    quat_to_2x2(g, h);
    for (int k = 0; k < 3; ++k) {
        cplx ik = h[0][0] * M->e[i][k] + h[0][1] * M->e[j][k];
        cplx jk = h[1][0] * M->e[i][k] + h[1][1] * M->e[j][k];
        M->e[i][k] = ik;
        M->e[j][k] = jk;
    }
}

/* columns i,j of M <- columns i,j times g^dag */
static void right_subgroup_mult_dag(mat3 *M, int i, int j, quat g) {
    cplx h[2][2];
    quat_to_2x2(g, h);
    for (int k = 0; k < 3; ++k) {
        cplx ki = M->e[k][i] * conj(h[0][0]) + M->e[k][j] * conj(h[0][1]);
        cplx kj = M->e[k][i] * conj(h[1][0]) + M->e[k][j] * conj(h[1][1]);
        M->e[k][i] = ki;
        M->e[k][j] = kj;
    }
}

/* quaternion product a*b, taken as the 2x2 matrix product */
static quat quat_mul(quat a, quat b) {
    cplx A[2][2], B[2][2], C[2][2];
    quat_to_2x2(a, A);
    quat_to_2x2(b, B);
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) C[r][c] = A[r][0] * B[0][c] + A[r][1] * B[1][c];
    quat q;
    q.v[0] = creal(C[0][0]);
    q.v[3] = cimag(C[0][0]);
    q.v[2] = creal(C[0][1]);
    q.v[1] = cimag(C[0][1]);
    return q;
}

static quat quat_unit(void) {
    quat q = {{1.0, 0.0, 0.0, 0.0}};
    return q;
}

/* App. A, Fig. calculateUpdate: first-order g -> g^omega (Sec. 2.2.3) */
static quat or_map(quat a, double omega) {
    double ai_sq = a.v[1] * a.v[1] + a.v[2] * a.v[2] + a.v[3] * a.v[3];
    double a0_sq = a.v[0] * a.v[0];
    double b = (omega * a0_sq + ai_sq) / (a0_sq + ai_sq);
    double c = 1.0 / sqrt(a0_sq + b * b * ai_sq);
    quat g;
    g.v[0] = a.v[0] * c;
    g.v[1] = a.v[1] * b * c;
    g.v[2] = a.v[2] * b * c;
    g.v[3] = a.v[3] * b * c;
    return g;
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11: Random123), as published        */
/* ------------------------------------------------------------------ */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void gfo_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, &hi0, &lo0);
        mulhilo64(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* 53-bit uniform strictly inside (0,1) */
static double u01(uint64_t w) { return ((double)(w >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

typedef struct {
    uint64_t key[2];   /* (seed, instance) */
    uint64_t sweep;    /* global sweep index */
    uint64_t site;     /* natural lexicographic site index */
    int subgroup;      /* 0,1,2 */
} rng_site;

/* four uniforms for (draw block, stream) of one site/subgroup */
static void draw4(const rng_site *r, uint64_t block, uint64_t stream, double u[4]) {
    uint64_t ctr[4] = {r->sweep, r->site, ((uint64_t)r->subgroup << 16) | block, stream};
    uint64_t out[4];
    gfo_philox4x64_10(ctr, r->key, out);
    for (int k = 0; k < 4; ++k) u[k] = u01(out[k]);
}

/* ------------------------------------------------------------------ */
/* Heatbath samplers (reading R10)                                     */
/* ------------------------------------------------------------------ */

/* w in [-1,1] with density ~ exp(kappa w): inverse of the CDF */
double gfo_exp_inverse_cdf(double kappa, double u) {
    if (kappa <= 0.0) return 2.0 * u - 1.0;
    /* w = 1 + log(exp(-2k) + u (1 - exp(-2k))) / k, written with expm1/log1p */
    double e = -expm1(-2.0 * kappa); /* 1 - exp(-2k) */
    return 1.0 + log1p(-(1.0 - u) * e) / kappa;
}

/* r0 with density ~ sqrt(1-r0^2) exp(a r0); returns the number of tries */
double gfo_sample_r0(double a, const uint64_t key[2], uint64_t sweep, uint64_t site, int subgroup, int *tries) {
    rng_site r = {{key[0], key[1]}, sweep, site, subgroup};
    double u[4];
    for (int t = 0; t < 64; ++t) {
        draw4(&r, (uint64_t)t, 0, u);
        if (a < 2.0) {
            /* Creutz: r0 from exp(a r0) by inverse CDF, accept with sqrt(1-r0^2) */
            double r0 = gfo_exp_inverse_cdf(a, u[0]);
            if (u[1] * u[1] <= 1.0 - r0 * r0) {
                if (tries) *tries = t + 1;
                return r0;
            }
        } else {
            /* Kennedy-Pendleton: lambda^2 ~ Gamma(3/2, rate 2a), accept with sqrt(1-lambda^2) */
            double c = cos(2.0 * M_PI * u[1]);
            double l2 = -(log(u[0]) + c * c * log(u[2])) / (2.0 * a);
            if (u[3] * u[3] <= 1.0 - l2) {
                if (tries) *tries = t + 1;
                return 1.0 - 2.0 * l2;
            }
        }
    }
    if (tries) *tries = 65;
    return 1.0;
}

/* ------------------------------------------------------------------ */
/* Local update, Step 1 of Alg. 1                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    int gauge;
    int update;
    double omega;
    double T;
    double p_sr;
    uint64_t key[2];
    uint64_t sweep;
} upd_params;

static const int SUB_I[3] = {0, 0, 1};
static const int SUB_J[3] = {1, 2, 2};

/* Landau/Coulomb relaxation direction: conj(q)/|q| (eq. localsolution) */
static quat landau_relax(quat q) {
    double n = sqrt(q.v[0] * q.v[0] + q.v[1] * q.v[1] + q.v[2] * q.v[2] + q.v[3] * q.v[3]);
    if (n == 0.0) return quat_unit();
    quat h = {{q.v[0] / n, -q.v[1] / n, -q.v[2] / n, -q.v[3] / n}};
    return h;
}

typedef struct { double D, E, F; } mag_coef;

/* MAG: coefficients of the local quadratic form (Sec. 2.2.2) for block (i,j),
   written with SU(3) block elements (reading R4). fwd[k]: U_mu(x),
   bwd[k]: U_mu(x - mu). */
static mag_coef mag_coefficients(const mat3 *fwd, const mat3 *bwd, int ndir, int i, int j) {
    mag_coef c = {0, 0, 0};
    for (int k = 0; k < ndir; ++k) {
        cplx a = fwd[k].e[i][i], b = fwd[k].e[i][j], cc = fwd[k].e[j][i], d = fwd[k].e[j][j];
        double aa = creal(a * conj(a)), bb = creal(b * conj(b)), c2 = creal(cc * conj(cc)), dd = creal(d * conj(d));
        c.D += 0.5 * (aa + dd - bb - c2);
        cplx w = a * conj(cc) - b * conj(d);
        c.F += creal(w);
        c.E += cimag(w);
    }
    for (int k = 0; k < ndir; ++k) {
        cplx a = bwd[k].e[i][i], b = bwd[k].e[i][j], cc = bwd[k].e[j][i], d = bwd[k].e[j][j];
        double aa = creal(a * conj(a)), bb = creal(b * conj(b)), c2 = creal(cc * conj(cc)), dd = creal(d * conj(d));
        c.D += 0.5 * (aa + dd - bb - c2);
        cplx w = conj(a) * b - d * conj(cc);
        c.F += creal(w);
        c.E += cimag(w);
    }
    return c;
}

/* MAG relaxation: eigenvector (D + lambda, E, F) of the largest eigenvalue */
static quat mag_relax(mag_coef c) {
    double lam = sqrt(c.D * c.D + c.E * c.E + c.F * c.F);
    if (lam == 0.0) return quat_unit();
    double g0 = c.D + lam, g1 = c.E, g2 = c.F;
    double n = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
    if (n == 0.0) {
        quat h = {{0.0, 1.0, 0.0, 0.0}};
        return h;
    }
    quat h = {{g0 / n, g1 / n, g2 / n, 0.0}};
    return h;
}

/* MAG heatbath: n ~ exp(kappa n.yhat) on S^2, then g (g3 = 0) with n(g) = n */
static quat mag_heatbath(mag_coef c, double T, const rng_site *r) {
    double y[3] = {c.F, -c.E, c.D};
    double lam = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    double u[4];
    draw4(r, 0, 0, u);
    double yh[3];
    if (lam == 0.0) {
        yh[0] = 0.0;
        yh[1] = 0.0;
        yh[2] = 1.0;
    } else {
        for (int k = 0; k < 3; ++k) yh[k] = y[k] / lam;
    }
    double kappa = lam / T;
    double w = gfo_exp_inverse_cdf(kappa, u[0]);
    double phi = 2.0 * M_PI * u[1];
    double s = sqrt(fmax(0.0, 1.0 - w * w));
    double e1[3], e2[3];
    double opz = 1.0 + yh[2];
    if (opz > 0.0) {
        e1[0] = 1.0 - yh[0] * yh[0] / opz;
        e1[1] = -yh[0] * yh[1] / opz;
        e1[2] = -yh[0];
        e2[0] = -yh[0] * yh[1] / opz;
        e2[1] = 1.0 - yh[1] * yh[1] / opz;
        e2[2] = -yh[1];
    } else {
        e1[0] = 1.0;
        e1[1] = 0.0;
        e1[2] = 0.0;
        e2[0] = 0.0;
        e2[1] = -1.0;
        e2[2] = 0.0;
    }
    double n[3];
    for (int k = 0; k < 3; ++k) n[k] = w * yh[k] + s * (cos(phi) * e1[k] + sin(phi) * e2[k]);
    double g0 = sqrt(fmax(0.0, 0.5 * (1.0 + n[2])));
    if (g0 == 0.0) {
        quat h = {{0.0, 1.0, 0.0, 0.0}};
        return h;
    }
    quat g = {{g0, -n[1] / (2.0 * g0), n[0] / (2.0 * g0), 0.0}};
    /* renormalise against rounding in n */
    double nn = sqrt(g.v[0] * g.v[0] + g.v[1] * g.v[1] + g.v[2] * g.v[2]);
    for (int k = 0; k < 4; ++k) g.v[k] /= nn;
    return g;
}

/* Landau/Coulomb heatbath: g = r * h, r0 from sqrt(1-r0^2) exp(|q| r0 / T) */
static quat landau_heatbath(quat q, double T, const rng_site *r) {
    double nq = sqrt(q.v[0] * q.v[0] + q.v[1] * q.v[1] + q.v[2] * q.v[2] + q.v[3] * q.v[3]);
    quat h = landau_relax(q);
    double a = nq / T;
    double r0 = gfo_sample_r0(a, r->key, r->sweep, r->site, r->subgroup, NULL);
    double u[4];
    draw4(r, 0, 1, u);
    double ct = 2.0 * u[0] - 1.0;
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double phi = 2.0 * M_PI * u[1];
    double rr = sqrt(fmax(0.0, 1.0 - r0 * r0));
    quat rq = {{r0, rr * st * cos(phi), rr * st * sin(phi), rr * ct}};
    return quat_mul(rq, h);
}

/* the final g from the relaxation direction h (and the update type) */
static quat finish_update(quat h, const upd_params *P, const rng_site *r) {
    switch (P->update) {
    case GFO_OR:
        return or_map(h, P->omega);
    case GFO_MICRO:
        return quat_mul(h, h);
    case GFO_SR: {
        double u[4];
        draw4(r, 0, 2, u);
        if (u[0] < P->p_sr) return quat_mul(h, h);
        return h;
    }
    default:
        return h;
    }
}

/* One full site update: three subgroups, each Step 1 then Step 2. */
static void update_site(double *U, double *G, const geom *g, int64_t s, const upd_params *P) {
    const int coulomb = (P->gauge == GFO_COULOMB);
    const int mu0 = coulomb ? 1 : 0;
    const int ndir = 4 - mu0;
    int64_t back[4];
    for (int mu = mu0; mu < 4; ++mu) back[mu] = site_shift(g, s, mu, -1);

    for (int sg = 0; sg < 3; ++sg) {
        const int i = SUB_I[sg], j = SUB_J[sg];
        mat3 fwd[4], bwd[4];
        for (int k = 0; k < ndir; ++k) {
            fwd[k] = link_get(U, s, mu0 + k);
            bwd[k] = link_get(U, back[mu0 + k], mu0 + k);
        }
        rng_site r = {{P->key[0], P->key[1]}, P->sweep, (uint64_t)s, sg};
        quat gq;
        if (P->gauge == GFO_MAG) {
            mag_coef c = mag_coefficients(fwd, bwd, ndir, i, j);
            if (P->update == GFO_HEATBATH)
                gq = mag_heatbath(c, P->T, &r);
            else
                gq = finish_update(mag_relax(c), P, &r);
        } else {
            /* K(x) = sum_mu U_mu(x) + U_mu(x - mu)^dag (eq. Kx, g's already applied) */
            mat3 K = mat_zero();
            for (int k = 0; k < ndir; ++k) {
                mat_acc(&K, &fwd[k]);
                mat3 bd = mat_dag(&bwd[k]);
                mat_acc(&K, &bd);
            }
            quat q = subgroup_quaternion(&K, i, j);
            if (P->update == GFO_HEATBATH)
                gq = landau_heatbath(q, P->T, &r);
            else
                gq = finish_update(landau_relax(q), P, &r);
        }
        /* Step 2: apply g to the adjacent links */
        for (int k = 0; k < ndir; ++k) {
            left_subgroup_mult(&fwd[k], i, j, gq);
            right_subgroup_mult_dag(&bwd[k], i, j, gq);
            link_put(U, s, mu0 + k, &fwd[k]);
            link_put(U, back[mu0 + k], mu0 + k, &bwd[k]);
        }
        if (coulomb && G) {
            mat3 Gx = mat_get18(G + (size_t)s * 18);
            left_subgroup_mult(&Gx, i, j, gq);
            mat_put18(G + (size_t)s * 18, &Gx);
        }
    }
}

static int site_active(const geom *g, int64_t s, int gauge, int parity, const uint8_t *slice_active) {
    if (gauge == GFO_COULOMB) {
        if (site_parity3(g, s) != parity) return 0;
        if (slice_active && !slice_active[site_t(g, s)]) return 0;
        return 1;
    }
    return site_parity4(g, s) == parity;
}

/* One half-sweep: every site of one parity (sites of one parity touch
   disjoint link sets, so their order does not matter). */
void gfo_halfsweep(double *U, const int32_t dims[4], int32_t gauge, int32_t update, int32_t parity, double omega,
                   double T, double p_sr, uint64_t seed, uint64_t instance, uint64_t sweep, double *G,
                   const uint8_t *slice_active) {
    geom g = make_geom(dims);
    upd_params P = {gauge, update, omega, T, p_sr, {seed, instance}, sweep};
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s)
        if (site_active(&g, s, gauge, parity, slice_active)) update_site(U, G, &g, s, &P);
}

void gfo_sweep(double *U, const int32_t dims[4], int32_t gauge, int32_t update, double omega, double T, double p_sr,
               uint64_t seed, uint64_t instance, uint64_t sweep, double *G, const uint8_t *slice_active) {
    for (int p = 0; p < 2; ++p)
        gfo_halfsweep(U, dims, gauge, update, p, omega, T, p_sr, seed, instance, sweep, G, slice_active);
}

/* Update an explicit list of sites, in list order (for sampled checks). */
void gfo_update_sites(double *U, const int32_t dims[4], int32_t gauge, int32_t update, double omega, double T,
                      double p_sr, uint64_t seed, uint64_t instance, uint64_t sweep, double *G, const int64_t *sites,
                      int64_t nsites) {
    geom g = make_geom(dims);
    upd_params P = {gauge, update, omega, T, p_sr, {seed, instance}, sweep};
    for (int64_t k = 0; k < nsites; ++k) update_site(U, G, &g, sites[k], &P);
}

/* Step 1 alone on explicit links (for unit tests): fwd/bwd are ndir links in
   the 18-real layout; returns the SU(2) element for subgroup (i,j). */
void gfo_local_g(const double *fwd18, const double *bwd18, int32_t ndir, int32_t gauge, int32_t update, int32_t i,
                 int32_t j, double omega, double T, double p_sr, uint64_t seed, uint64_t instance, uint64_t sweep,
                 uint64_t site, int32_t subgroup, double out[4]) {
    mat3 fwd[4], bwd[4];
    for (int k = 0; k < ndir; ++k) {
        fwd[k] = mat_get18(fwd18 + 18 * k);
        bwd[k] = mat_get18(bwd18 + 18 * k);
    }
    upd_params P = {gauge, update, omega, T, p_sr, {seed, instance}, sweep};
    rng_site r = {{seed, instance}, sweep, site, subgroup};
    quat gq;
    if (gauge == GFO_MAG) {
        mag_coef c = mag_coefficients(fwd, bwd, ndir, i, j);
        gq = (update == GFO_HEATBATH) ? mag_heatbath(c, T, &r) : finish_update(mag_relax(c), &P, &r);
    } else {
        mat3 K = mat_zero();
        for (int k = 0; k < ndir; ++k) {
            mat_acc(&K, &fwd[k]);
            mat3 bd = mat_dag(&bwd[k]);
            mat_acc(&K, &bd);
        }
        quat q = subgroup_quaternion(&K, i, j);
        gq = (update == GFO_HEATBATH) ? landau_heatbath(q, T, &r) : finish_update(landau_relax(q), &P, &r);
    }
    for (int k = 0; k < 4; ++k) out[k] = gq.v[k];
}

/* MAG coefficients (D, E, F) for unit tests */
void gfo_mag_coefficients(const double *fwd18, const double *bwd18, int32_t ndir, int32_t i, int32_t j,
                          double out[3]) {
    mat3 fwd[4], bwd[4];
    for (int k = 0; k < ndir; ++k) {
        fwd[k] = mat_get18(fwd18 + 18 * k);
        bwd[k] = mat_get18(bwd18 + 18 * k);
    }
    mag_coef c = mag_coefficients(fwd, bwd, ndir, i, j);
    out[0] = c.D;
    out[1] = c.E;
    out[2] = c.F;
}

/* exported algebra for the printed-code checks */
void gfo_subgroup_quaternion(const double *M18, int32_t i, int32_t j, double out[4]) {
    mat3 M = mat_get18(M18);
    quat q = subgroup_quaternion(&M, i, j);
    for (int k = 0; k < 4; ++k) out[k] = q.v[k];
}

void gfo_left_subgroup_mult(double *M18, int32_t i, int32_t j, const double g[4]) {
    mat3 M = mat_get18(M18);
    quat q = {{g[0], g[1], g[2], g[3]}};
    left_subgroup_mult(&M, i, j, q);
    mat_put18(M18, &M);
}

void gfo_right_subgroup_mult_dag(double *M18, int32_t i, int32_t j, const double g[4]) {
    mat3 M = mat_get18(M18);
    quat q = {{g[0], g[1], g[2], g[3]}};
    right_subgroup_mult_dag(&M, i, j, q);
    mat_put18(M18, &M);
}

void gfo_or_map(const double a[4], double omega, double out[4]) {
    quat q = {{a[0], a[1], a[2], a[3]}};
    quat g = or_map(q, omega);
    for (int k = 0; k < 4; ++k) out[k] = g.v[k];
}

void gfo_quat_mul(const double a[4], const double b[4], double out[4]) {
    quat qa = {{a[0], a[1], a[2], a[3]}}, qb = {{b[0], b[1], b[2], b[3]}};
    quat r = quat_mul(qa, qb);
    for (int k = 0; k < 4; ++k) out[k] = r.v[k];
}

/* ------------------------------------------------------------------ */
/* Functionals and gauge precision (Sec. 2.1)                          */
/* ------------------------------------------------------------------ */

/* Landau: F = (1/(Nc Nd V)) Re sum tr U;  theta = (1/(Nc V)) sum tr Delta Delta^dag,
   Delta(x) = sum_mu A_mu(x) - A_mu(x - mu).
   MAG: F = (1/(Nc Nd V)) sum |U_ii|^2; theta per reading R8. */
void gfo_measure(const double *U, const int32_t dims[4], int32_t gauge, double *F_out, double *theta_out) {
    geom g = make_geom(dims);
    const int mu0 = (gauge == GFO_COULOMB) ? 1 : 0;
    const int ndir = 4 - mu0;
    double Fs = 0.0, Ts = 0.0;
#pragma omp parallel for reduction(+ : Fs, Ts) schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        if (gauge == GFO_MAG) {
            mat3 W = mat_zero();
            for (int mu = 0; mu < 4; ++mu) {
                mat3 u = link_get(U, s, mu);
                for (int i = 0; i < 3; ++i) Fs += creal(u.e[i][i] * conj(u.e[i][i]));
                mat3 ub = link_get(U, site_shift(&g, s, mu, -1), mu);
                /* U diag(U)^dag - diag(U')^dag U' */
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        W.e[i][j] += u.e[i][j] * conj(u.e[j][j]) - conj(ub.e[i][i]) * ub.e[i][j];
            }
            double t = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = i + 1; j < 3; ++j) {
                    cplx gam = W.e[i][j] - conj(W.e[j][i]);
                    t += creal(gam * conj(gam));
                }
            Ts += t;
        } else {
            mat3 Delta = mat_zero();
            for (int mu = mu0; mu < 4; ++mu) {
                mat3 u = link_get(U, s, mu);
                Fs += mat_retrace(&u);
                mat3 ub = link_get(U, site_shift(&g, s, mu, -1), mu);
                mat3 A = mat_antiherm_traceless(&u);
                mat3 Ab = mat_antiherm_traceless(&ub);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) Delta.e[i][j] += A.e[i][j] - Ab.e[i][j];
            }
            Ts += mat_norm2(&Delta);
        }
    }
    *F_out = Fs / (3.0 * ndir * (double)g.V);
    *theta_out = Ts / (3.0 * (double)g.V);
}

/* Coulomb: per time-slice F_t and theta_t (reading R9) */
void gfo_measure_slices(const double *U, const int32_t dims[4], double *F_t, double *theta_t) {
    geom g = make_geom(dims);
    const int64_t Nt = g.n[0];
    const int64_t Vs = g.V / Nt;
    for (int64_t t = 0; t < Nt; ++t) {
        double Fs = 0.0, Ts = 0.0;
#pragma omp parallel for reduction(+ : Fs, Ts) schedule(static)
        for (int64_t k = 0; k < Vs; ++k) {
            int64_t s = t * Vs + k;
            mat3 Delta = mat_zero();
            for (int mu = 1; mu < 4; ++mu) {
                mat3 u = link_get(U, s, mu);
                Fs += mat_retrace(&u);
                mat3 ub = link_get(U, site_shift(&g, s, mu, -1), mu);
                mat3 A = mat_antiherm_traceless(&u);
                mat3 Ab = mat_antiherm_traceless(&ub);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) Delta.e[i][j] += A.e[i][j] - Ab.e[i][j];
            }
            Ts += mat_norm2(&Delta);
        }
        F_t[t] = Fs / (9.0 * (double)Vs);
        theta_t[t] = Ts / (3.0 * (double)Vs);
    }
}

/* Identity check helper: Delta(x) = [(K - K^dag)/(2i)]_traceless, with
   K(x) = sum_mu U_mu(x) + U_mu(x - mu)^dag.  Returns theta computed that way. */
double gfo_theta_via_K(const double *U, const int32_t dims[4], int32_t gauge) {
    geom g = make_geom(dims);
    const int mu0 = (gauge == GFO_COULOMB) ? 1 : 0;
    double Ts = 0.0;
#pragma omp parallel for reduction(+ : Ts) schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        mat3 K = mat_zero();
        for (int mu = mu0; mu < 4; ++mu) {
            mat3 u = link_get(U, s, mu);
            mat3 ub = link_get(U, site_shift(&g, s, mu, -1), mu);
            mat3 ubd = mat_dag(&ub);
            mat_acc(&K, &u);
            mat_acc(&K, &ubd);
        }
        mat3 D = mat_antiherm_traceless(&K);
        Ts += mat_norm2(&D);
    }
    return Ts / (3.0 * (double)g.V);
}

/* Identity check helper: MAG theta from the subgroup coefficients,
   sum over subgroups of E^2 + F^2 (the squared subgroup gradient). */
double gfo_theta_mag_via_subgroups(const double *U, const int32_t dims[4]) {
    geom g = make_geom(dims);
    double Ts = 0.0;
#pragma omp parallel for reduction(+ : Ts) schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        mat3 fwd[4], bwd[4];
        for (int mu = 0; mu < 4; ++mu) {
            fwd[mu] = link_get(U, s, mu);
            bwd[mu] = link_get(U, site_shift(&g, s, mu, -1), mu);
        }
        for (int sg = 0; sg < 3; ++sg) {
            mag_coef c = mag_coefficients(fwd, bwd, 4, SUB_I[sg], SUB_J[sg]);
            Ts += c.E * c.E + c.F * c.F;
        }
    }
    return Ts / (3.0 * (double)g.V);
}

/* MAG theta in the literal squared-sum form of Sec. 2.1.2 (reported only;
   parity unpinned: the printed form is ambiguous and nothing depends on it) */
double gfo_theta_mag_literal(const double *U, const int32_t dims[4]) {
    geom g = make_geom(dims);
    double Ts = 0.0;
#pragma omp parallel for reduction(+ : Ts) schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        mat3 W = mat_zero();
        for (int mu = 0; mu < 4; ++mu) {
            mat3 u = link_get(U, s, mu);
            mat3 ub = link_get(U, site_shift(&g, s, mu, -1), mu);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) W.e[i][j] += u.e[i][j] * conj(u.e[j][j]) - conj(ub.e[i][i]) * ub.e[i][j];
        }
        cplx sum = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = i + 1; j < 3; ++j) sum += W.e[i][j] - conj(W.e[j][i]);
        Ts += creal(sum * conj(sum));
    }
    return Ts / (3.0 * (double)g.V);
}

/* Unitarity monitor (Sec. 4.5): mean and max |1 - det U| over nlinks links */
void gfo_unitarity(const double *U, int64_t nlinks, double *mean, double *maxv) {
    double s = 0.0, m = 0.0;
#pragma omp parallel for reduction(+ : s) reduction(max : m) schedule(static)
    for (int64_t l = 0; l < nlinks; ++l) {
        mat3 u = mat_get18(U + (size_t)l * 18);
        double d = cabs(1.0 - mat_det(&u));
        s += d;
        if (d > m) m = d;
    }
    *mean = s / (double)nlinks;
    *maxv = m;
}

/* max over links of |U U^dag - 1| (Frobenius), a stricter unitarity check */
double gfo_unitarity_defect(const double *U, int64_t nlinks) {
    double m = 0.0;
#pragma omp parallel for reduction(max : m) schedule(static)
    for (int64_t l = 0; l < nlinks; ++l) {
        mat3 u = mat_get18(U + (size_t)l * 18);
        mat3 ud = mat_dag(&u);
        mat3 p = mat_mul(&u, &ud);
        for (int i = 0; i < 3; ++i) p.e[i][i] -= 1.0;
        double d = sqrt(mat_norm2(&p));
        if (d > m) m = d;
    }
    return m;
}

void gfo_reunitarise(double *U, int64_t nlinks) {
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < nlinks; ++l) {
        mat3 u = mat_get18(U + (size_t)l * 18);
        mat_reunitarise(&u);
        mat_put18(U + (size_t)l * 18, &u);
    }
}

/* ------------------------------------------------------------------ */
/* Gauge invariants: plaquette and rectangular Wilson loops            */
/* ------------------------------------------------------------------ */

/* product of n links starting at s along +mu; *end receives the end site */
static mat3 line_product(const double *U, const geom *g, int64_t s, int mu, int n, int64_t *end) {
    mat3 P = mat_identity();
    for (int k = 0; k < n; ++k) {
        mat3 u = link_get(U, s, mu);
        P = mat_mul(&P, &u);
        s = site_shift(g, s, mu, +1);
    }
    *end = s;
    return P;
}

/* average of (1/3) Re tr of the R x T loop over all sites and all ordered
   planes (mu != nu), R links along mu and T along nu */
double gfo_wilson_loop(const double *U, const int32_t dims[4], int32_t R, int32_t Tt) {
    geom g = make_geom(dims);
    double s_all = 0.0;
#pragma omp parallel for reduction(+ : s_all) schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = 0; nu < 4; ++nu) {
                if (mu == nu) continue;
                int64_t a, b, c, d;
                mat3 L1 = line_product(U, &g, s, mu, R, &a);  /* s -> s+R mu */
                mat3 L2 = line_product(U, &g, a, nu, Tt, &b); /* -> s+R mu+T nu */
                mat3 L3 = line_product(U, &g, s, nu, Tt, &c); /* s -> s+T nu */
                mat3 L4 = line_product(U, &g, c, mu, R, &d);  /* -> s+T nu+R mu */
                mat3 A = mat_mul(&L1, &L2);
                mat3 B = mat_mul(&L3, &L4);
                mat3 Bd = mat_dag(&B);
                mat3 W = mat_mul(&A, &Bd);
                s_all += mat_retrace(&W) / 3.0;
            }
    }
    return s_all / (12.0 * (double)g.V);
}

double gfo_plaquette(const double *U, const int32_t dims[4]) { return gfo_wilson_loop(U, dims, 1, 1); }

/* U_mu(x) <- g(x) U_mu(x) g(x+mu)^dag for a site field g (V x 18 reals) */
void gfo_apply_gauge(double *U, const int32_t dims[4], const double *gfield) {
    geom g = make_geom(dims);
    double *out = (double *)malloc(sizeof(double) * 18 * 4 * (size_t)g.V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        mat3 gx = mat_get18(gfield + (size_t)s * 18);
        for (int mu = 0; mu < 4; ++mu) {
            mat3 gy = mat_get18(gfield + (size_t)site_shift(&g, s, mu, +1) * 18);
            mat3 gyd = mat_dag(&gy);
            mat3 u = link_get(U, s, mu);
            mat3 t = mat_mul(&gx, &u);
            mat3 r = mat_mul(&t, &gyd);
            mat_put18(out + ((size_t)s * 4 + mu) * 18, &r);
        }
    }
    memcpy(U, out, sizeof(double) * 18 * 4 * (size_t)g.V);
    free(out);
}

/* Coulomb finish (reading R9): U_0(x) <- G(x) U_0(x) G(x+0)^dag */
void gfo_coulomb_fix_u0(double *U, const int32_t dims[4], const double *G) {
    geom g = make_geom(dims);
    double *u0 = (double *)malloc(sizeof(double) * 18 * (size_t)g.V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        mat3 gx = mat_get18(G + (size_t)s * 18);
        mat3 gy = mat_get18(G + (size_t)site_shift(&g, s, 0, +1) * 18);
        mat3 gyd = mat_dag(&gy);
        mat3 u = link_get(U, s, 0);
        mat3 t = mat_mul(&gx, &u);
        mat3 r = mat_mul(&t, &gyd);
        mat_put18(u0 + (size_t)s * 18, &r);
    }
    for (int64_t s = 0; s < g.V; ++s) {
        mat3 r = mat_get18(u0 + (size_t)s * 18);
        link_put(U, s, 0, &r);
    }
    free(u0);
}

/* ------------------------------------------------------------------ */
/* Alg. 1 driver with the stopping rule                                */
/* ------------------------------------------------------------------ */

/* Runs sweeps of one update type until theta < tol at a check (checks after
   every check_every sweeps, and once on the input) or max_sweeps.
   Landau/MAG: one instance; Coulomb: every time-slice stops on its own and
   the U_0 fix-up is applied at the end.
   traj_F/traj_theta (may be NULL) receive the measured values at each check,
   traj_sweep the sweep count at that check; *ntraj the number of checks
   recorded (at most traj_cap).  sweeps_done: one entry (Landau/MAG) or Nt
   entries (Coulomb).  *sweep_counter is the global sweep index, advanced by
   the number of sweeps run (used for random streams).
   reunit_every > 0: after every reunit_every sweeps reproject the links of
   the instance, or (Coulomb) the links and the accumulated transformation of
   every time-slice still running (reading R13).
   Returns 0 if converged, 1 if some instance/slice hit max_sweeps. */
int gfo_run(double *U, const int32_t dims[4], int32_t gauge, int32_t update, double omega, double p_sr,
            int32_t max_sweeps, double tol, int32_t check_every, int32_t reunit_every, uint64_t seed,
            uint64_t instance, uint64_t *sweep_counter, int64_t *sweeps_done, double *traj_F, double *traj_theta,
            int32_t *traj_sweep, int32_t traj_cap, int32_t *ntraj) {
    geom g = make_geom(dims);
    const int64_t Nt = g.n[0];
    int n = 0;
    int status = 0;
    if (check_every < 1) check_every = 1;
    if (gauge == GFO_COULOMB) {
        double *G = (double *)malloc(sizeof(double) * 18 * (size_t)g.V);
        for (int64_t s = 0; s < g.V; ++s) {
            mat3 id = mat_identity();
            mat_put18(G + (size_t)s * 18, &id);
        }
        uint8_t *active = (uint8_t *)malloc((size_t)Nt);
        double *Ft = (double *)malloc(sizeof(double) * (size_t)Nt);
        double *Tt = (double *)malloc(sizeof(double) * (size_t)Nt);
        for (int64_t t = 0; t < Nt; ++t) {
            active[t] = 1;
            sweeps_done[t] = 0;
        }
        int k = 0;
        for (;;) {
            if (k % check_every == 0) {
                gfo_measure_slices(U, dims, Ft, Tt);
                double Fm = 0, Tm = 0;
                for (int64_t t = 0; t < Nt; ++t) {
                    Fm += Ft[t];
                    Tm += Tt[t];
                    if (active[t] && Tt[t] < tol) active[t] = 0;
                }
                if (traj_F && n < traj_cap) {
                    traj_F[n] = Fm / (double)Nt;
                    traj_theta[n] = Tm / (double)Nt;
                    traj_sweep[n] = k;
                    ++n;
                }
            }
            int any = 0;
            for (int64_t t = 0; t < Nt; ++t) any |= active[t];
            if (!any) break;
            if (k >= max_sweeps) {
                status = 1;
                break;
            }
            gfo_sweep(U, dims, gauge, update, omega, 0.0, p_sr, seed, instance, *sweep_counter, G, active);
            ++*sweep_counter;
            ++k;
            for (int64_t t = 0; t < Nt; ++t)
                if (active[t]) sweeps_done[t] = k;
            if (reunit_every > 0 && k % reunit_every == 0) {
                /* R13: the four links and the accumulated transformation of
                   every site of a time-slice still running */
#pragma omp parallel for schedule(static)
                for (int64_t s = 0; s < g.V; ++s) {
                    if (!active[site_t(&g, s)]) continue;
                    for (int mu = 0; mu < 4; ++mu) {
                        mat3 u = link_get(U, s, mu);
                        mat_reunitarise(&u);
                        link_put(U, s, mu, &u);
                    }
                    mat3 gs = mat_get18(G + (size_t)s * 18);
                    mat_reunitarise(&gs);
                    mat_put18(G + (size_t)s * 18, &gs);
                }
            }
        }
        gfo_coulomb_fix_u0(U, dims, G);
        free(G);
        free(active);
        free(Ft);
        free(Tt);
    } else {
        int k = 0;
        sweeps_done[0] = 0;
        for (;;) {
            if (k % check_every == 0) {
                double F, th;
                gfo_measure(U, dims, gauge, &F, &th);
                if (traj_F && n < traj_cap) {
                    traj_F[n] = F;
                    traj_theta[n] = th;
                    traj_sweep[n] = k;
                    ++n;
                }
                if (th < tol) break;
            }
            if (k >= max_sweeps) {
                status = 1;
                break;
            }
            gfo_sweep(U, dims, gauge, update, omega, 0.0, p_sr, seed, instance, *sweep_counter, NULL, NULL);
            ++*sweep_counter;
            ++k;
            sweeps_done[0] = k;
            if (reunit_every > 0 && k % reunit_every == 0) gfo_reunitarise(U, 4 * g.V);
        }
    }
    if (ntraj) *ntraj = n;
    return status;
}

/* Simulated annealing (Sec. 2.3, reading R11): for k = 0..nsteps-1,
   T_k = T0 + (T1 - T0) k / (nsteps - 1); one heatbath sweep at T_k, then
   nmicro microcanonical sweeps.  Coulomb accumulates into G (V x 18, may be
   NULL for Landau/MAG). *sweep_counter advances by every sweep run. */
void gfo_anneal(double *U, const int32_t dims[4], int32_t gauge, double T0, double T1, int32_t nsteps, int32_t nmicro,
                uint64_t seed, uint64_t instance, uint64_t *sweep_counter, double *G) {
    for (int k = 0; k < nsteps; ++k) {
        double T = (nsteps > 1) ? T0 + (T1 - T0) * (double)k / (double)(nsteps - 1) : T0;
        gfo_sweep(U, dims, gauge, GFO_HEATBATH, 1.0, T, 0.0, seed, instance, *sweep_counter, G, NULL);
        ++*sweep_counter;
        for (int m = 0; m < nmicro; ++m) {
            gfo_sweep(U, dims, gauge, GFO_MICRO, 1.0, 0.0, 0.0, seed, instance, *sweep_counter, G, NULL);
            ++*sweep_counter;
        }
    }
}

/* ================================================================== */
/* SU(2) gauge group (N_c = 2): Sec. 2.1 and 2.2 for SU(2) itself       */
/* ================================================================== */
/*
 * Links are 2x2 complex matrices in the natural layout
 * (sites, 4, 2, 2, re/im), 8 reals per link.  The local update is done on
 * the whole group, with no subgroup iteration:
 *   Landau/Coulomb: K(x) = sum_mu U_mu(x) + U_mu(x - mu)^dag and the optimum
 *     g = K^dag / sqrt(det K^dag) (eq. localsolution, written out as matrices);
 *   MAG: the coefficients D, E, F of the quadratic form of eq. upMatrix in
 *     the Cayley-Klein components of the links (reading R4: D twice the
 *     printed value, written without using det U = 1).  The backward link
 *     transforms as U_mu(x - mu) g(x)^dag, so its term is the forward term
 *     of U_mu(x - mu)^dag (reading R12);
 *   overrelaxation, microcanonical and stochastic relaxation steps and both
 *     heatbaths as for one SU(3) subgroup (readings R5, R6, R10), with the
 *     random counter's subgroup field 0;
 *   F and theta as in Sec. 2.1 with N_c = 2: the MAG theta from the
 *     off-diagonal element of X(x) of Sec. 2.1.2, computed as matrices.
 */

typedef struct { cplx e[2][2]; } mat2;

static mat2 m2_get(const double *p) {
    mat2 m;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) m.e[i][j] = CMPLX(p[2 * (2 * i + j)], p[2 * (2 * i + j) + 1]);
    return m;
}

static void m2_put(double *p, const mat2 *m) {
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            p[2 * (2 * i + j)] = creal(m->e[i][j]);
            p[2 * (2 * i + j) + 1] = cimag(m->e[i][j]);
        }
}

static mat2 l2_get(const double *U, int64_t s, int mu) { return m2_get(U + ((size_t)s * 4 + mu) * 8); }
static void l2_put(double *U, int64_t s, int mu, const mat2 *m) { m2_put(U + ((size_t)s * 4 + mu) * 8, m); }

static mat2 m2_zero(void) {
    mat2 m;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) m.e[i][j] = 0.0;
    return m;
}

static mat2 m2_mul(const mat2 *a, const mat2 *b) {
    mat2 c;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) c.e[i][j] = a->e[i][0] * b->e[0][j] + a->e[i][1] * b->e[1][j];
    return c;
}

static mat2 m2_dag(const mat2 *a) {
    mat2 c;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) c.e[i][j] = conj(a->e[j][i]);
    return c;
}

static cplx m2_det(const mat2 *a) { return a->e[0][0] * a->e[1][1] - a->e[0][1] * a->e[1][0]; }

/* Cayley-Klein components of an SU(2) matrix (from its first row) */
static quat m2_quat(const mat2 *m) {
    quat q;
    q.v[0] = creal(m->e[0][0]);
    q.v[3] = cimag(m->e[0][0]);
    q.v[2] = creal(m->e[0][1]);
    q.v[1] = cimag(m->e[0][1]);
    return q;
}

static mat2 quat_m2(quat g) {
    mat2 m;
    quat_to_2x2(g, m.e);
    return m;
}

/* traceless part of (M - M^dag)/(2i) (reading R7 for N_c = 2) */
static mat2 m2_antiherm_traceless(const mat2 *m) {
    mat2 a;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) a.e[i][j] = (m->e[i][j] - conj(m->e[j][i])) / (2.0 * I);
    cplx tr = (a.e[0][0] + a.e[1][1]) / 2.0;
    a.e[0][0] -= tr;
    a.e[1][1] -= tr;
    return a;
}

static double m2_norm2(const mat2 *a) {
    double s = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) s += creal(a->e[i][j] * conj(a->e[i][j]));
    return s;
}

/* the printed MAG coefficients of one link (D doubled, reading R4) */
static void su2_mag_add(quat u, mag_coef *c) {
    c->D += u.v[0] * u.v[0] + u.v[3] * u.v[3] - u.v[1] * u.v[1] - u.v[2] * u.v[2];
    c->E += 2.0 * (-u.v[0] * u.v[1] - u.v[2] * u.v[3]);
    c->F += 2.0 * (-u.v[0] * u.v[2] + u.v[1] * u.v[3]);
}

/* Step 1 for SU(2): the g(x) of the update, from the adjacent links */
static mat2 su2_local(const mat2 *fwd, const mat2 *bwd, int ndir, const upd_params *P, const rng_site *r) {
    quat gq;
    if (P->gauge == GFO_MAG) {
        mag_coef c = {0, 0, 0};
        for (int k = 0; k < ndir; ++k) su2_mag_add(m2_quat(&fwd[k]), &c);
        for (int k = 0; k < ndir; ++k) {
            mat2 bd = m2_dag(&bwd[k]);
            su2_mag_add(m2_quat(&bd), &c);
        }
        if (P->update == GFO_HEATBATH)
            gq = mag_heatbath(c, P->T, r);
        else
            gq = finish_update(mag_relax(c), P, r);
        return quat_m2(gq);
    }
    mat2 K = m2_zero();
    for (int k = 0; k < ndir; ++k) {
        mat2 bd = m2_dag(&bwd[k]);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) K.e[i][j] += fwd[k].e[i][j] + bd.e[i][j];
    }
    mat2 Kd = m2_dag(&K);
    cplx det = m2_det(&Kd);
    mat2 h;
    if (det == 0.0) {
        h = quat_m2(quat_unit());
    } else {
        cplx sq = csqrt(det);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) h.e[i][j] = Kd.e[i][j] / sq;
    }
    quat hq = m2_quat(&h);
    if (P->update == GFO_HEATBATH) {
        /* g = r h, r0 ~ sqrt(1 - r0^2) exp(a r0) with a T = Re tr[h K], the
           local functional at the optimum (reading R10) */
        mat2 hK = m2_mul(&h, &K);
        double a = creal(hK.e[0][0] + hK.e[1][1]) / P->T;
        double r0 = gfo_sample_r0(a, r->key, r->sweep, r->site, r->subgroup, NULL);
        double u[4];
        draw4(r, 0, 1, u);
        double ct = 2.0 * u[0] - 1.0;
        double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        double phi = 2.0 * M_PI * u[1];
        double rr = sqrt(fmax(0.0, 1.0 - r0 * r0));
        quat rq = {{r0, rr * st * cos(phi), rr * st * sin(phi), rr * ct}};
        mat2 rm = quat_m2(rq);
        return m2_mul(&rm, &h);
    }
    if (P->update == GFO_MICRO) return m2_mul(&h, &h);
    if (P->update == GFO_SR) {
        double u[4];
        draw4(r, 0, 2, u);
        if (u[0] < P->p_sr) return m2_mul(&h, &h);
        return h;
    }
    return quat_m2(or_map(hq, P->omega));
}

/* one SU(2) site update: Step 1, then Step 2 on the adjacent links */
static void su2_update_site(double *U, double *G, const geom *g, int64_t s, const upd_params *P) {
    const int coulomb = (P->gauge == GFO_COULOMB);
    const int mu0 = coulomb ? 1 : 0;
    const int ndir = 4 - mu0;
    int64_t back[4];
    mat2 fwd[4], bwd[4];
    for (int k = 0; k < ndir; ++k) {
        back[k] = site_shift(g, s, mu0 + k, -1);
        fwd[k] = l2_get(U, s, mu0 + k);
        bwd[k] = l2_get(U, back[k], mu0 + k);
    }
    rng_site r = {{P->key[0], P->key[1]}, P->sweep, (uint64_t)s, 0};
    mat2 gx = su2_local(fwd, bwd, ndir, P, &r);
    mat2 gd = m2_dag(&gx);
    for (int k = 0; k < ndir; ++k) {
        mat2 f = m2_mul(&gx, &fwd[k]);
        mat2 b = m2_mul(&bwd[k], &gd);
        l2_put(U, s, mu0 + k, &f);
        l2_put(U, back[k], mu0 + k, &b);
    }
    if (coulomb && G) {
        mat2 Gx = m2_get(G + (size_t)s * 8);
        mat2 n = m2_mul(&gx, &Gx);
        m2_put(G + (size_t)s * 8, &n);
    }
}

void gfo2_halfsweep(double *U, const int32_t dims[4], int32_t gauge, int32_t update, int32_t parity, double omega,
                    double T, double p_sr, uint64_t seed, uint64_t instance, uint64_t sweep, double *G,
                    const uint8_t *slice_active) {
    geom g = make_geom(dims);
    upd_params P = {gauge, update, omega, T, p_sr, {seed, instance}, sweep};
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s)
        if (site_active(&g, s, gauge, parity, slice_active)) su2_update_site(U, G, &g, s, &P);
}

void gfo2_update_sites(double *U, const int32_t dims[4], int32_t gauge, int32_t update, double omega, double T,
                       double p_sr, uint64_t seed, uint64_t instance, uint64_t sweep, double *G,
                       const int64_t *sites, int64_t nsites) {
    geom g = make_geom(dims);
    upd_params P = {gauge, update, omega, T, p_sr, {seed, instance}, sweep};
    for (int64_t k = 0; k < nsites; ++k) su2_update_site(U, G, &g, sites[k], &P);
}

/* Step 1 alone on explicit links (unit tests): fwd/bwd are ndir links of 8
   reals; out receives g(x) as 8 reals */
void gfo2_local_g(const double *fwd8, const double *bwd8, int32_t ndir, int32_t gauge, int32_t update, double omega,
                  double T, double p_sr, uint64_t seed, uint64_t instance, uint64_t sweep, uint64_t site,
                  double out[8]) {
    mat2 fwd[4], bwd[4];
    for (int k = 0; k < ndir; ++k) {
        fwd[k] = m2_get(fwd8 + 8 * k);
        bwd[k] = m2_get(bwd8 + 8 * k);
    }
    upd_params P = {gauge, update, omega, T, p_sr, {seed, instance}, sweep};
    rng_site r = {{seed, instance}, sweep, site, 0};
    mat2 gx = su2_local(fwd, bwd, ndir, &P, &r);
    m2_put(out, &gx);
}

/* per-site F and theta contributions (Sec. 2.1, N_c = 2) */
static void su2_site_measure(const double *U, const geom *g, int64_t s, int gauge, double *F, double *T) {
    const int mu0 = (gauge == GFO_COULOMB) ? 1 : 0;
    if (gauge == GFO_MAG) {
        /* X(x) = sum_mu U sigma3 U^dag + U'^dag sigma3 U' (Sec. 2.1.2) */
        mat2 s3 = m2_zero();
        s3.e[0][0] = 1.0;
        s3.e[1][1] = -1.0;
        mat2 X = m2_zero();
        for (int mu = 0; mu < 4; ++mu) {
            mat2 u = l2_get(U, s, mu);
            for (int i = 0; i < 2; ++i) *F += creal(u.e[i][i] * conj(u.e[i][i]));
            mat2 ub = l2_get(U, site_shift(g, s, mu, -1), mu);
            mat2 ud = m2_dag(&u), ubd = m2_dag(&ub);
            mat2 t1 = m2_mul(&u, &s3), a = m2_mul(&t1, &ud);
            mat2 t2 = m2_mul(&ubd, &s3), b = m2_mul(&t2, &ub);
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) X.e[i][j] += a.e[i][j] + b.e[i][j];
        }
        *T += creal(X.e[0][1] * conj(X.e[0][1]));
        return;
    }
    mat2 Delta = m2_zero();
    for (int mu = mu0; mu < 4; ++mu) {
        mat2 u = l2_get(U, s, mu);
        *F += creal(u.e[0][0] + u.e[1][1]);
        mat2 ub = l2_get(U, site_shift(g, s, mu, -1), mu);
        mat2 A = m2_antiherm_traceless(&u), Ab = m2_antiherm_traceless(&ub);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) Delta.e[i][j] += A.e[i][j] - Ab.e[i][j];
    }
    *T += m2_norm2(&Delta);
}

/* F = (1/(N_c N_d V)) sum (Re tr U | sum_i |U_ii|^2), theta = (1/(N_c V)) sum ... */
void gfo2_measure(const double *U, const int32_t dims[4], int32_t gauge, double *F_out, double *theta_out) {
    geom g = make_geom(dims);
    const int ndir = (gauge == GFO_COULOMB) ? 3 : 4;
    double Fs = 0.0, Ts = 0.0;
#pragma omp parallel for reduction(+ : Fs, Ts) schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        double f = 0.0, t = 0.0;
        su2_site_measure(U, &g, s, gauge, &f, &t);
        Fs += f;
        Ts += t;
    }
    *F_out = Fs / (2.0 * ndir * (double)g.V);
    *theta_out = Ts / (2.0 * (double)g.V);
}

/* Coulomb: per time-slice F_t and theta_t */
void gfo2_measure_slices(const double *U, const int32_t dims[4], double *F_t, double *theta_t) {
    geom g = make_geom(dims);
    const int64_t Nt = g.n[0], Vs = g.V / Nt;
    for (int64_t t = 0; t < Nt; ++t) {
        double Fs = 0.0, Ts = 0.0;
#pragma omp parallel for reduction(+ : Fs, Ts) schedule(static)
        for (int64_t k = 0; k < Vs; ++k) {
            double f = 0.0, th = 0.0;
            su2_site_measure(U, &g, t * Vs + k, GFO_COULOMB, &f, &th);
            Fs += f;
            Ts += th;
        }
        F_t[t] = Fs / (6.0 * (double)Vs);
        theta_t[t] = Ts / (2.0 * (double)Vs);
    }
}

/* mean and max |1 - det U| over nlinks links */
void gfo2_unitarity(const double *U, int64_t nlinks, double *mean, double *maxv) {
    double s = 0.0, m = 0.0;
    for (int64_t k = 0; k < nlinks; ++k) {
        mat2 u = m2_get(U + 8 * (size_t)k);
        double e = cabs(1.0 - m2_det(&u));
        s += e;
        if (e > m) m = e;
    }
    *mean = nlinks ? s / (double)nlinks : 0.0;
    *maxv = m;
}

/* reprojection to SU(2): normalise row 0, row 1 = (-conj(b), conj(a)) */
void gfo2_reunitarise(double *U, int64_t nlinks) {
    for (int64_t k = 0; k < nlinks; ++k) {
        mat2 u = m2_get(U + 8 * (size_t)k);
        double n = sqrt(creal(u.e[0][0] * conj(u.e[0][0]) + u.e[0][1] * conj(u.e[0][1])));
        u.e[0][0] /= n;
        u.e[0][1] /= n;
        u.e[1][0] = -conj(u.e[0][1]);
        u.e[1][1] = conj(u.e[0][0]);
        m2_put(U + 8 * (size_t)k, &u);
    }
}

/* average of (1/2) Re tr of the 1x1 plaquettes over all sites and planes */
double gfo2_plaquette(const double *U, const int32_t dims[4]) {
    geom g = make_geom(dims);
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t x = 0; x < g.V; ++x)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                mat2 a = l2_get(U, x, mu), b = l2_get(U, site_shift(&g, x, mu, +1), nu);
                mat2 c = l2_get(U, site_shift(&g, x, nu, +1), mu), d = l2_get(U, x, nu);
                mat2 cd = m2_dag(&c), dd = m2_dag(&d);
                mat2 ab = m2_mul(&a, &b), abc = m2_mul(&ab, &cd), p = m2_mul(&abc, &dd);
                s += 0.5 * creal(p.e[0][0] + p.e[1][1]);
            }
    return s / (6.0 * (double)g.V);
}

/* U_mu(x) <- g(x) U_mu(x) g(x + mu)^dag for a site field g (V x 8 reals) */
void gfo2_apply_gauge(double *U, const int32_t dims[4], const double *gfield) {
    geom g = make_geom(dims);
    double *out = (double *)malloc(sizeof(double) * 32 * (size_t)g.V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        mat2 gx = m2_get(gfield + (size_t)s * 8);
        for (int mu = 0; mu < 4; ++mu) {
            mat2 gy = m2_get(gfield + (size_t)site_shift(&g, s, mu, +1) * 8);
            mat2 gyd = m2_dag(&gy), u = l2_get(U, s, mu);
            mat2 t = m2_mul(&gx, &u), r = m2_mul(&t, &gyd);
            m2_put(out + ((size_t)s * 4 + mu) * 8, &r);
        }
    }
    memcpy(U, out, sizeof(double) * 32 * (size_t)g.V);
    free(out);
}

/* Coulomb finish for SU(2) (reading R9): U_0(x) <- G(x) U_0(x) G(x+0)^dag */
void gfo2_coulomb_fix_u0(double *U, const int32_t dims[4], const double *G) {
    geom g = make_geom(dims);
    double *u0 = (double *)malloc(sizeof(double) * 8 * (size_t)g.V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        mat2 gx = m2_get(G + (size_t)s * 8);
        mat2 gy = m2_get(G + (size_t)site_shift(&g, s, 0, +1) * 8);
        mat2 gyd = m2_dag(&gy), u = l2_get(U, s, 0);
        mat2 t = m2_mul(&gx, &u), r = m2_mul(&t, &gyd);
        m2_put(u0 + (size_t)s * 8, &r);
    }
    for (int64_t s = 0; s < g.V; ++s) {
        mat2 r = m2_get(u0 + (size_t)s * 8);
        l2_put(U, s, 0, &r);
    }
    free(u0);
}
