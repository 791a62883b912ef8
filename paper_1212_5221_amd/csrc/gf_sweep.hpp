// gf_sweep.hpp -- the half-sweep kernel of Alg. 1 (one parity of every
// active unit), templated on gauge, update type, link storage, compute
// precision and the number W of wavefronts that share a group of 64 sites.
//
// Per site x of the active parity (Sec. 2.4, Alg. 1):
//   1. load the adjacent links U_mu(x) and U_mu(x - mu) (8, Coulomb 6);
//   2. for the SU(2) subgroups (0,1), (0,2), (1,2) compute the local g
//      (Step 1) from the links with the previous subgroups' g applied;
//   3. apply the product G = g3 g2 g1 to the links once (Step 2) and store.
// Applying g1, g2, g3 one after the other to the links equals applying G:
// the same update as the paper's, with the links loaded and stored once and
// one 3x3 product per link instead of three subgroup products.
// Landau/Coulomb: K(x) = sum_mu U_mu(x) + U_mu(x - mu)^dag becomes g K after
// the subgroup step, so K is summed once and updated in registers
// (eq. Kx with the g(x + mu) already absorbed in the stored links).
// MAG: the 2x2 blocks of G U_mu(x) and U_mu(x - mu) G^dag give the
// quadratic-form coefficients of each subgroup (Sec. 2.2.2, with the
// coefficient D twice the printed value so that the matrix form agrees with
// the explicit form).
#pragma once

#include <type_traits>

#include "gf_device.hpp"

namespace gfd {


// ---------------------------------------------------------------- updates
template <typename T>
__device__ __forceinline__ Q4<T> q_unit() {
    Q4<T> g;
    g.v[0] = T(1);
    g.v[1] = g.v[2] = g.v[3] = T(0);
    return g;
}

// subgroup quaternion of the 2x2 block (i,j) (App. A)
template <typename T>
__device__ __forceinline__ Q4<T> block_quat(const M3<T> &K, int i, int j) {
    Q4<T> q;
    q.v[0] = K.e[i][i].re + K.e[j][j].re;
    q.v[3] = K.e[i][i].im - K.e[j][j].im;
    q.v[2] = K.e[i][j].re - K.e[j][i].re;
    q.v[1] = K.e[i][j].im + K.e[j][i].im;
    return q;
}

// maximum of Re tr[g K]: the conjugate of q, normalised (eq. localsolution)
template <typename T>
__device__ __forceinline__ Q4<T> landau_relax(const Q4<T> &q) {
    const T n2 = q.v[0] * q.v[0] + q.v[1] * q.v[1] + q.v[2] * q.v[2] + q.v[3] * q.v[3];
    if (n2 == T(0)) return q_unit<T>();
    const T inv = T(1) / sqrt(n2);
    Q4<T> h;
    h.v[0] = q.v[0] * inv;
    h.v[1] = -q.v[1] * inv;
    h.v[2] = -q.v[2] * inv;
    h.v[3] = -q.v[3] * inv;
    return h;
}

// top eigenvector (D + lambda, E, F) of the MAG quadratic form
template <typename T>
__device__ __forceinline__ Q4<T> mag_relax(T D, T E, T F) {
    const T lam = sqrt(D * D + E * E + F * F);
    if (lam == T(0)) return q_unit<T>();
    const T g0 = D + lam;
    const T n2 = g0 * g0 + E * E + F * F;
    Q4<T> h;
    if (n2 == T(0)) {
        h.v[0] = T(0);
        h.v[1] = T(1);
        h.v[2] = h.v[3] = T(0);
        return h;
    }
    const T inv = T(1) / sqrt(n2);
    h.v[0] = g0 * inv;
    h.v[1] = E * inv;
    h.v[2] = F * inv;
    h.v[3] = T(0);
    return h;
}

// first-order g -> g^omega (App. A, overrelaxation update)
template <typename T>
__device__ __forceinline__ Q4<T> or_map(const Q4<T> &a, T omega) {
    const T ai2 = a.v[1] * a.v[1] + a.v[2] * a.v[2] + a.v[3] * a.v[3];
    const T a02 = a.v[0] * a.v[0];
    const T b = (omega * a02 + ai2) / (a02 + ai2);
    const T c = T(1) / sqrt(a02 + b * b * ai2);
    Q4<T> g;
    g.v[0] = a.v[0] * c;
    g.v[1] = a.v[1] * (b * c);
    g.v[2] = a.v[2] * (b * c);
    g.v[3] = a.v[3] * (b * c);
    return g;
}

// w in [-1, 1] with density ~ exp(kappa w), by inverting the CDF
__device__ __forceinline__ double exp_icdf(double kappa, double u) {
    if (kappa <= 0.0) return 2.0 * u - 1.0;
    const double e = -expm1(-2.0 * kappa);
    return 1.0 + log1p(-(1.0 - u) * e) / kappa;
}

// r0 with density ~ sqrt(1 - r0^2) exp(a r0): Creutz (a < 2) or
// Kennedy-Pendleton (a >= 2), at most 64 tries
__device__ __forceinline__ double sample_r0(double a, const Rng &rng) {
    double u[4];
    for (int t = 0; t < 64; ++t) {
        rng.draw((uint64_t)t, 0, u);
        if (a < 2.0) {
            const double r0 = exp_icdf(a, u[0]);
            if (u[1] * u[1] <= 1.0 - r0 * r0) return r0;
        } else {
            const double c = cos(2.0 * M_PI * u[1]);
            const double l2 = -(log(u[0]) + c * c * log(u[2])) / (2.0 * a);
            if (u[3] * u[3] <= 1.0 - l2) return 1.0 - 2.0 * l2;
        }
    }
    return 1.0;
}

// Landau/Coulomb heatbath: g = r h with r0 ~ sqrt(1 - r0^2) exp(|q| r0 / T)
__device__ __forceinline__ Q4<double> landau_heatbath(const Q4<double> &q, double T, const Rng &rng) {
    const double nq = sqrt(q.v[0] * q.v[0] + q.v[1] * q.v[1] + q.v[2] * q.v[2] + q.v[3] * q.v[3]);
    const Q4<double> h = landau_relax(q);
    const double r0 = sample_r0(nq / T, rng);
    double u[4];
    rng.draw(0, 1, u);
    const double ct = 2.0 * u[0] - 1.0;
    const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    const double phi = 2.0 * M_PI * u[1];
    const double rr = sqrt(fmax(0.0, 1.0 - r0 * r0));
    Q4<double> r;
    r.v[0] = r0;
    r.v[1] = rr * st * cos(phi);
    r.v[2] = rr * st * sin(phi);
    r.v[3] = rr * ct;
    return qmul(r, h);
}

// MAG heatbath: n(g) from von Mises-Fisher exp(kappa n.yhat), y = (F, -E, D),
// kappa = lambda / T; then g (g3 = 0) with n(g) = n
// u0, u1: the first two uniforms of the subgroup's draw (block 0, stream 0)
__device__ __forceinline__ Q4<double> mag_heatbath(double D, double E, double F, double T, double u0, double u1) {
    double y0 = F, y1 = -E, y2 = D;
    const double lam = sqrt(y0 * y0 + y1 * y1 + y2 * y2);
    if (lam == 0.0) {
        y0 = 0.0;
        y1 = 0.0;
        y2 = 1.0;
    } else {
        y0 /= lam;
        y1 /= lam;
        y2 /= lam;
    }
    const double w = exp_icdf(lam / T, u0);
    const double phi = 2.0 * M_PI * u1;
    const double s = sqrt(fmax(0.0, 1.0 - w * w));
    double e1[3], e2[3];
    const double opz = 1.0 + y2;
    if (opz > 0.0) {
        e1[0] = 1.0 - y0 * y0 / opz;
        e1[1] = -y0 * y1 / opz;
        e1[2] = -y0;
        e2[0] = -y0 * y1 / opz;
        e2[1] = 1.0 - y1 * y1 / opz;
        e2[2] = -y1;
    } else {
        e1[0] = 1.0;
        e1[1] = 0.0;
        e1[2] = 0.0;
        e2[0] = 0.0;
        e2[1] = -1.0;
        e2[2] = 0.0;
    }
    const double cp = cos(phi), sp = sin(phi);
    const double n0 = w * y0 + s * (cp * e1[0] + sp * e2[0]);
    const double n1 = w * y1 + s * (cp * e1[1] + sp * e2[1]);
    const double n2 = w * y2 + s * (cp * e1[2] + sp * e2[2]);
    const double g0 = sqrt(fmax(0.0, 0.5 * (1.0 + n2)));
    Q4<double> g;
    if (g0 == 0.0) {
        g.v[0] = 0.0;
        g.v[1] = 1.0;
        g.v[2] = g.v[3] = 0.0;
        return g;
    }
    g.v[0] = g0;
    g.v[1] = -n1 / (2.0 * g0);
    g.v[2] = n0 / (2.0 * g0);
    g.v[3] = 0.0;
    const double nn = sqrt(g.v[0] * g.v[0] + g.v[1] * g.v[1] + g.v[2] * g.v[2]);
    g.v[0] /= nn;
    g.v[1] /= nn;
    g.v[2] /= nn;
    return g;
}

template <typename T>
__device__ __forceinline__ Q4<T> to_T(const Q4<double> &g) {
    Q4<T> r;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.v[k] = T(g.v[k]);
    return r;
}

template <typename T>
__device__ __forceinline__ Q4<double> to_d(const Q4<T> &g) {
    Q4<double> r;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.v[k] = double(g.v[k]);
    return r;
}

// relaxation direction h -> the applied g for OR / micro / SR
template <int UPD, typename T>
__device__ __forceinline__ Q4<T> finish(const Q4<T> &h, const gfs::SweepArgs &a, const Rng &rng) {
    if constexpr (UPD == gfs::UPD_OR) return or_map(h, T(a.omega));
    if constexpr (UPD == gfs::UPD_MICRO) return qmul(h, h);
    if constexpr (UPD == gfs::UPD_SR) {
        double u[4];
        rng.draw(0, 2, u);
        if (u[0] < a.p_sr) return qmul(h, h);
        return h;
    }
    return h;
}

// The W waves of a site group hold the same K (or MAG coefficients), so a
// heatbath sample, which costs Philox draws, transcendental functions and a
// rejection loop, is drawn by wave 0 alone and handed to the others through
// LDS (one slot per subgroup, so one barrier per subgroup suffices).
template <int W, int GROUPS, typename T>
__device__ __forceinline__ void share_from_wave0(Q4<T> &g, int sg, int grp, int wv, int lane) {
    if constexpr (W > 1) {
        __shared__ T shg[3][GROUPS][4][64];
        if (wv == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) shg[sg][grp][k][lane] = g.v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) g.v[k] = shg[sg][grp][k][lane];
    }
}

// ---------------------------------------------------------------- MAG blocks
// block (i,j) of G U (forward link) and of U G^dag (backward link)
// G is the product of the subgroup elements of the earlier subgroups: the
// identity before subgroup 0, and nontrivial only in its (0,1) block before
// subgroup 1.  The block products below skip those known zeros, which the
// compiler has to keep (x * 0 is not 0 for x = NaN or -0).
template <typename T>
__device__ __forceinline__ void mag_coef_add(cx<T> a, cx<T> b, cx<T> c, cx<T> d, bool fwd, T &D, T &E, T &F) {
    D += T(0.5) * (cnorm2(a) + cnorm2(d) - cnorm2(b) - cnorm2(c));
    const cx<T> w = fwd ? csub(cmulc(a, c), cmulc(b, d))   // a c* - b d*
                        : csub(cmulc(b, a), cmulc(d, c));  // a* b - d c*
    F += w.re;
    E += w.im;
}

// block (i,j) of G U (forward link), subgroup SG
template <int SG, typename T>
__device__ __forceinline__ void mag_block_fwd(const M3<T> &G, const M3<T> &U, T &D, T &E, T &F) {
    constexpr int i = (SG == 2) ? 1 : 0, j = (SG == 0) ? 1 : 2;
    cx<T> a, b, c, d;
    if constexpr (SG == 0) {
        a = U.e[0][0];
        b = U.e[0][1];
        c = U.e[1][0];
        d = U.e[1][1];
    } else if constexpr (SG == 1) {
        a = cmac(cmul(G.e[0][0], U.e[0][0]), G.e[0][1], U.e[1][0]);
        b = cmac(cmul(G.e[0][0], U.e[0][2]), G.e[0][1], U.e[1][2]);
        c = U.e[2][0];
        d = U.e[2][2];
    } else {
        a = cmul(G.e[i][0], U.e[0][i]);
        b = cmul(G.e[i][0], U.e[0][j]);
        c = cmul(G.e[j][0], U.e[0][i]);
        d = cmul(G.e[j][0], U.e[0][j]);
#pragma unroll
        for (int k = 1; k < 3; ++k) {
            a = cmac(a, G.e[i][k], U.e[k][i]);
            b = cmac(b, G.e[i][k], U.e[k][j]);
            c = cmac(c, G.e[j][k], U.e[k][i]);
            d = cmac(d, G.e[j][k], U.e[k][j]);
        }
    }
    mag_coef_add(a, b, c, d, true, D, E, F);
}

// block (i,j) of U G^dag (backward link), subgroup SG
template <int SG, typename T>
__device__ __forceinline__ void mag_block_bwd(const M3<T> &G, const M3<T> &U, T &D, T &E, T &F) {
    constexpr int i = (SG == 2) ? 1 : 0, j = (SG == 0) ? 1 : 2;
    cx<T> a, b, c, d;
    if constexpr (SG == 0) {
        a = U.e[0][0];
        b = U.e[0][1];
        c = U.e[1][0];
        d = U.e[1][1];
    } else if constexpr (SG == 1) {
        a = cmacc(cmulc(U.e[0][0], G.e[0][0]), U.e[0][1], G.e[0][1]);
        b = U.e[0][2];
        c = cmacc(cmulc(U.e[2][0], G.e[0][0]), U.e[2][1], G.e[0][1]);
        d = U.e[2][2];
    } else {
        a = cmulc(U.e[i][0], G.e[i][0]);
        b = cmulc(U.e[i][0], G.e[j][0]);
        c = cmulc(U.e[j][0], G.e[i][0]);
        d = cmulc(U.e[j][0], G.e[j][0]);
#pragma unroll
        for (int k = 1; k < 3; ++k) {
            a = cmacc(a, U.e[i][k], G.e[i][k]);
            b = cmacc(b, U.e[i][k], G.e[j][k]);
            c = cmacc(c, U.e[j][k], G.e[i][k]);
            d = cmacc(d, U.e[j][k], G.e[j][k]);
        }
    }
    mag_coef_add(a, b, c, d, false, D, E, F);
}

// ---------------------------------------------------------------- apply
// rows 0..ROWS-1 of G U
template <typename T>
__device__ __forceinline__ void apply_left(const M3<T> &G, const M3<T> &U, M3<T> &out, int rows) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (i >= rows) break;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmul(G.e[i][0], U.e[0][j]);
            s = cmac(s, G.e[i][1], U.e[1][j]);
            s = cmac(s, G.e[i][2], U.e[2][j]);
            out.e[i][j] = s;
        }
    }
}

// rows 0..ROWS-1 of U G^dag (needs only those rows of U)
template <typename T>
__device__ __forceinline__ void apply_right_dag(const M3<T> &G, const M3<T> &U, M3<T> &out, int rows) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (i >= rows) break;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmulc(U.e[i][0], G.e[j][0]);
            s = cmacc(s, U.e[i][1], G.e[j][1]);
            s = cmacc(s, U.e[i][2], G.e[j][2]);
            out.e[i][j] = s;
        }
    }
}

// ---------------------------------------------------------------- kernel
// BLK threads per block (BLK / (64 W) site groups); NT: non-temporal loads
// and stores of the links (streaming past the caches, for lattices larger
// than the Infinity Cache)
template <int GAUGE, int UPD, int ST, typename CT, int W, int BLK, int NT>
__global__ __launch_bounds__(BLK) void k_sweep(gfs::SweepArgs a) {
    typedef Store<ST> SD;
    typedef typename SD::S S;
    typedef typename SD::V V;
    constexpr int NDIR = (GAUGE == gfs::COULOMB) ? 3 : 4;
    constexpr int MU0 = (GAUGE == gfs::COULOMB) ? 1 : 0;
    constexpr int NL = 2 * NDIR;
    constexpr int LPW = NL / W;
    static_assert(NL % W == 0, "waves must split the links evenly");
    constexpr int GROUPS = BLK / (64 * W);
    static_assert(GROUPS >= 1, "block too small");

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wv = wave % W, grp = wave / W;
    const gfs::Tile tl = a.tiles[a.xcd_order ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x];
    const int u = tl.unit;
    if (!a.active[u]) return;
    if (a.fp64_select >= 0 && a.fp64[u] != a.fp64_select) return;
    const gfs::UnitDev U = a.unit[u];
    const gfs::InstDev I = a.inst[U.inst];

    int32_t j = tl.j0 + grp * 64 + lane;
    const bool valid = j < U.n;
    if (!valid) j = U.n - 1;  // keep every lane on a real site; only valid lanes store
    const int32_t h = U.h0 + j;
    // storage (4D) parity of the active site; Coulomb selects by 3D parity
    const int p = (GAUGE == gfs::COULOMB) ? ((a.parity + U.t) & 1) : a.parity;
    const Site s = site_of(I, h, p);

    // ---- load this wave's links
    S r[LPW][SD::NR];
    int32_t lh[LPW];
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
        const int l = wv * LPW + q;
        const bool fw = l < NDIR;
        const int mu = MU0 + (fw ? l : l - NDIR);
        lh[q] = fw ? h : back_h(I, s, h, mu);
        SD::template load<NT != 0>(plane_ptr<ST>(a.ws, I, fw ? p : 1 - p, mu), I.Vh, lh[q], r[q]);
    }

    Rng rng;
    rng.k0 = a.seed;
    rng.k1 = (uint64_t)U.inst;
    rng.sweep = a.sweep_ix[U.inst] + (uint64_t)a.sweep_off;
    rng.site = (uint64_t)natural_index(I, s);

    M3<CT> G;
    m3_identity(G);

    if constexpr (GAUGE != gfs::MAG) {
        // K(x) = sum_mu U_mu(x) + U_mu(x - mu)^dag
        M3<CT> K;
        m3_zero(K);
#pragma unroll
        for (int q = 0; q < LPW; ++q) {
            const int l = wv * LPW + q;
            M3<CT> m;
            expand<ST, CT>(r[q], m);
            if (l < NDIR) {
#pragma unroll
                for (int i2 = 0; i2 < 3; ++i2)
#pragma unroll
                    for (int j2 = 0; j2 < 3; ++j2) K.e[i2][j2] = cadd(K.e[i2][j2], m.e[i2][j2]);
            } else {
#pragma unroll
                for (int i2 = 0; i2 < 3; ++i2)
#pragma unroll
                    for (int j2 = 0; j2 < 3; ++j2) K.e[i2][j2] = cadd(K.e[i2][j2], cconj(m.e[j2][i2]));
            }
        }
        if constexpr (W > 1) {
            __shared__ CT shk[GROUPS][W][18][64];
#pragma unroll
            for (int i2 = 0; i2 < 3; ++i2)
#pragma unroll
                for (int j2 = 0; j2 < 3; ++j2) {
                    shk[grp][wv][2 * (3 * i2 + j2)][lane] = K.e[i2][j2].re;
                    shk[grp][wv][2 * (3 * i2 + j2) + 1][lane] = K.e[i2][j2].im;
                }
            __syncthreads();
#pragma unroll
            for (int i2 = 0; i2 < 3; ++i2)
#pragma unroll
                for (int j2 = 0; j2 < 3; ++j2) {
                    CT re = CT(0), im = CT(0);
#pragma unroll
                    for (int w2 = 0; w2 < W; ++w2) {
                        re += shk[grp][w2][2 * (3 * i2 + j2)][lane];
                        im += shk[grp][w2][2 * (3 * i2 + j2) + 1][lane];
                    }
                    K.e[i2][j2] = cmk(re, im);
                }
        }
#pragma unroll
        for (int sg = 0; sg < 3; ++sg) {
            const int i = (sg == 2) ? 1 : 0, jj = (sg == 0) ? 1 : 2;
            const Q4<CT> q = block_quat(K, i, jj);
            rng.sg = (uint64_t)sg;
            Q4<CT> g;
            if constexpr (UPD == gfs::UPD_HEATBATH) {
                if (wv == 0) g = to_T<CT>(landau_heatbath(to_d(q), a.T, rng));
                share_from_wave0<W, GROUPS>(g, sg, grp, wv, lane);
            } else {
                g = finish<UPD, CT>(landau_relax(q), a, rng);
            }
            left_sub(K, i, jj, g);
            left_sub(G, i, jj, g);
        }
    } else {
        // MAG: coefficients of each subgroup from the blocks of the links
        // with the partial G applied
        double hb_u[3][2];
        if constexpr (UPD == gfs::UPD_HEATBATH) {
            // the heatbath's random numbers do not depend on the links: the
            // three subgroups' Philox chains are computed together, so they
            // interleave instead of running back to back
            if (wv == 0) {
#pragma unroll
                for (int sg = 0; sg < 3; ++sg) {
                    Rng r2 = rng;
                    r2.sg = (uint64_t)sg;
                    double u[4];
                    r2.draw(0, 0, u);
                    hb_u[sg][0] = u[0];
                    hb_u[sg][1] = u[1];
                }
            }
        }
#pragma unroll
        for (int sg = 0; sg < 3; ++sg) {
            const int i = (sg == 2) ? 1 : 0, jj = (sg == 0) ? 1 : 2;
            CT D = CT(0), E = CT(0), F = CT(0);
#pragma unroll
            for (int q = 0; q < LPW; ++q) {
                const int l = wv * LPW + q;
                M3<CT> m;
                expand<ST, CT>(r[q], m);
                if (l < NDIR) {
                    if (sg == 0)
                        mag_block_fwd<0>(G, m, D, E, F);
                    else if (sg == 1)
                        mag_block_fwd<1>(G, m, D, E, F);
                    else
                        mag_block_fwd<2>(G, m, D, E, F);
                } else {
                    if (sg == 0)
                        mag_block_bwd<0>(G, m, D, E, F);
                    else if (sg == 1)
                        mag_block_bwd<1>(G, m, D, E, F);
                    else
                        mag_block_bwd<2>(G, m, D, E, F);
                }
            }
            if constexpr (W > 1) {
                __shared__ CT shm[3][GROUPS][W][3][64];
                shm[sg][grp][wv][0][lane] = D;
                shm[sg][grp][wv][1][lane] = E;
                shm[sg][grp][wv][2][lane] = F;
                __syncthreads();
                D = E = F = CT(0);
#pragma unroll
                for (int w2 = 0; w2 < W; ++w2) {
                    D += shm[sg][grp][w2][0][lane];
                    E += shm[sg][grp][w2][1][lane];
                    F += shm[sg][grp][w2][2][lane];
                }
            }
            rng.sg = (uint64_t)sg;
            Q4<CT> g;
            if constexpr (UPD == gfs::UPD_HEATBATH) {
                if (wv == 0) g = to_T<CT>(mag_heatbath(double(D), double(E), double(F), a.T, hb_u[sg][0], hb_u[sg][1]));
                share_from_wave0<W, GROUPS>(g, sg, grp, wv, lane);
            } else {
                g = finish<UPD, CT>(mag_relax(D, E, F), a, rng);
            }
            left_sub(G, i, jj, g);
        }
    }

    // ---- Step 2: apply G to this wave's links and store.
    // The empty asm makes the stored rows opaque, so the compiler rebuilds
    // the third rows here instead of keeping all expanded links live.
    // Landau/Coulomb heatbath: K holds all the sampler needs, so the links
    // are read again for Step 2, one at a time, instead of being held
    // through the sampling; their registers are free while the sampler's
    // long dependent chains run, and more waves fit on a SIMD to hide them.
    // The second read mostly hits the caches.
    constexpr bool RELOAD = (UPD == gfs::UPD_HEATBATH) && (GAUGE != gfs::MAG);
    if constexpr (RELOAD) {
        asm volatile("" ::: "memory");
    } else {
#pragma unroll
        for (int q = 0; q < LPW; ++q)
#pragma unroll
            for (int c = 0; c < SD::NR; ++c) asm volatile("" : "+v"(r[q][c]));
    }
    // FP32 storage: G is applied in FP64, and a G built in FP32 is first
    // reprojected to SU(3) in FP64.  An exactly unitary G keeps the links on
    // their gauge orbit, so the only loss is the rounding of the stored links.
    typedef typename std::conditional<ST == gfs::ST_F32R12, double, CT>::type AT;
    M3<AT> Ga;
#pragma unroll
    for (int i2 = 0; i2 < 3; ++i2)
#pragma unroll
        for (int j2 = 0; j2 < 3; ++j2) Ga.e[i2][j2] = cmk<AT>(AT(G.e[i2][j2].re), AT(G.e[i2][j2].im));
    if constexpr (!std::is_same<AT, CT>::value) reproject(Ga);
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
        const int l = wv * LPW + q;
        const bool fw = l < NDIR;
        const int mu = MU0 + (fw ? l : l - NDIR);
        M3<AT> m, o;
        if constexpr (RELOAD) {
            SD::template load<NT != 0>(plane_ptr<ST>(a.ws, I, fw ? p : 1 - p, mu), I.Vh, lh[q], r[q]);
#pragma unroll
            for (int c = 0; c < SD::NR; ++c) asm volatile("" : "+v"(r[q][c]));
        }
        expand<ST, AT>(r[q], m);
        if (fw) {
            apply_left(Ga, m, o, SD::ROWS);
            if constexpr (SD::ROWS == 2) renormalise_rows(o);
        } else {
            apply_right_dag(Ga, m, o, SD::ROWS);
        }
        compress<ST, AT>(o, r[q]);
        if (valid) SD::template store<NT != 0>(plane_ptr<ST>(a.ws, I, fw ? p : 1 - p, mu), I.Vh, lh[q], r[q]);
    }

    // ---- Coulomb: accumulate G(x) <- G G(x) (wave 0 of the group)
    if constexpr (GAUGE == gfs::COULOMB) {
      if (wv == 0) {
        V *gp = gacc_ptr<ST>(a.ws, I, p);
        S gr[SD::NR];
        SD::template load<NT != 0>(gp, I.Vh, h, gr);
        M3<AT> m, o;
        expand<ST, AT>(gr, m);
        apply_left(Ga, m, o, SD::ROWS);
        if constexpr (SD::ROWS == 2) renormalise_rows(o);
        compress<ST, AT>(o, gr);
        if (valid) SD::template store<NT != 0>(gp, I.Vh, h, gr);
      }
    }
}

}  // namespace gfd
