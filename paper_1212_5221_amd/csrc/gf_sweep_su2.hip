// gf_sweep_su2.hip -- the gauge group SU(2): link storage as the 4 real
// Cayley-Klein components (Sec. 2.2.2), the half-sweep kernel whose local
// update acts on the whole group (Sec. 2.2.1 eq. localsolution, Sec. 2.2.2
// eq. upMatrix; no subgroup iteration), and the F / theta, reprojection,
// layout conversion and Coulomb kernels for that storage.
//
// A link U = [[u0 + i u3, u2 + i u1], [-u2 + i u1, u0 - i u3]] is stored as
// (u0, u1, u2, u3) in the parity-split block layout of the SU(3) storages:
// FP64 as two 16-byte chunks (u0, u1), (u2, u3); FP32 as one float4.  A site
// of the active parity reads and writes its 8 (Coulomb 6) links once:
// 256 bytes (FP32) or 512 bytes (FP64) of traffic per site update.
#include <array>
#include <type_traits>
#include <utility>

#include "gf_launch.hpp"
#include "gf_reduce.hpp"
#include "gf_sweep.hpp"
#include "gf_variants.hpp"

namespace gfd {

template <>
struct Store<gfs::ST_SU2_F64> {
    typedef double S;
    typedef double2 V;
    static constexpr int NR = 4, NCH = 2;
    __device__ static __forceinline__ void load(const V *__restrict__ base, int64_t, int64_t h, S r[NR]) {
        const V *sv = site_vec<NCH>(base, (uint32_t)h);
        const V a = sv[0], b = sv[16];
        r[0] = a.x;
        r[1] = a.y;
        r[2] = b.x;
        r[3] = b.y;
    }
    __device__ static __forceinline__ void store(V *__restrict__ base, int64_t, int64_t h, const S r[NR]) {
        V *sv = site_vec<NCH>(base, (uint32_t)h);
        sv[0] = make_double2(r[0], r[1]);
        sv[16] = make_double2(r[2], r[3]);
    }
};

template <>
struct Store<gfs::ST_SU2_F32> {
    typedef float S;
    typedef float4 V;
    static constexpr int NR = 4, NCH = 1;
    __device__ static __forceinline__ void load(const V *__restrict__ base, int64_t, int64_t h, S r[NR]) {
        const V a = *site_vec<NCH>(base, (uint32_t)h);
        r[0] = a.x;
        r[1] = a.y;
        r[2] = a.z;
        r[3] = a.w;
    }
    __device__ static __forceinline__ void store(V *__restrict__ base, int64_t, int64_t h, const S r[NR]) {
        *site_vec<NCH>(base, (uint32_t)h) = make_float4(r[0], r[1], r[2], r[3]);
    }
};

// single precision: the same storage, g applied in FP32
template <>
struct Store<gfs::ST_SU2_F32_SP> : Store<gfs::ST_SU2_F32> {};

template <typename T, typename S>
__device__ __forceinline__ Q4<T> q_from(const S r[4]) {
    Q4<T> q;
#pragma unroll
    for (int k = 0; k < 4; ++k) q.v[k] = T(r[k]);
    return q;
}

template <typename T>
__device__ __forceinline__ Q4<T> q_dag(const Q4<T> &a) {
    Q4<T> r;
    r.v[0] = a.v[0];
    r.v[1] = -a.v[1];
    r.v[2] = -a.v[2];
    r.v[3] = -a.v[3];
    return r;
}

template <typename T>
__device__ __forceinline__ void q_normalise(Q4<T> &a) {
    const T n = T(1) / sqrt(a.v[0] * a.v[0] + a.v[1] * a.v[1] + a.v[2] * a.v[2] + a.v[3] * a.v[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) a.v[k] *= n;
}

// MAG coefficients of one SU(2) link from its matrix elements (the block
// formula with G = 1: D twice the printed value)
template <typename T>
__device__ __forceinline__ void su2_mag_add(const Q4<T> &u, bool fwd, T &D, T &E, T &F) {
    mag_coef_add(cmk(u.v[0], u.v[3]), cmk(u.v[2], u.v[1]), cmk(-u.v[2], u.v[1]), cmk(u.v[0], -u.v[3]), fwd, D, E, F);
}

// ---------------------------------------------------------------- half-sweep
// One thread per site of the active parity (no wave split: the 8 links are
// 32 or 64 registers).  The local g is computed in CT; on FP32 storage it is
// normalised and applied in FP64 (single precision: applied in FP32).
template <int GAUGE, int UPD, int ST, typename CT, int BLK>
__global__ __launch_bounds__(BLK) void k_sweep_su2(gfs::SweepArgs a) {
    typedef Store<ST> SD;
    typedef typename SD::S S;
    typedef typename SD::V V;
    constexpr int NDIR = (GAUGE == gfs::COULOMB) ? 3 : 4;
    constexpr int MU0 = (GAUGE == gfs::COULOMB) ? 1 : 0;
    constexpr int NL = 2 * NDIR;

    const gfs::Tile tl = a.tiles[a.xcd_order ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x];
    const int u = tl.unit;
    if (!a.active[u]) return;
    if (a.fp64_select >= 0 && a.fp64[u] != a.fp64_select) return;
    const gfs::UnitDev U = a.unit[u];
    const gfs::InstDev I = a.inst[U.inst];

    int32_t j = tl.j0 + (int32_t)threadIdx.x;
    const bool valid = j < U.n;
    if (!valid) j = U.n - 1;
    const int32_t h = U.h0 + j;
    const int p = (GAUGE == gfs::COULOMB) ? ((a.parity + U.t) & 1) : a.parity;
    const Site s = site_of(I, h, p);

    S r[NL][4];
    int32_t lh[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const bool fw = l < NDIR;
        const int mu = MU0 + (fw ? l : l - NDIR);
        lh[l] = fw ? h : back_h(I, s, h, mu);
        SD::load(plane_ptr<ST>(a.ws, I, fw ? p : 1 - p, mu), I.Vh, lh[l], r[l]);
    }

    Rng rng;
    rng.k0 = a.seed;
    rng.k1 = (uint64_t)U.inst;
    rng.sweep = a.sweep_ix[U.inst] + (uint64_t)a.sweep_off;
    rng.site = (uint64_t)natural_index(I, s);
    rng.sg = 0;

    Q4<CT> g;
    if constexpr (GAUGE != gfs::MAG) {
        // K(x) = sum_mu U_mu(x) + U_mu(x - mu)^dag is a multiple of an SU(2)
        // matrix; q = 2 x its Cayley-Klein components (the quaternion of a
        // 2x2 block, so that Re tr[g K] = |q| at the optimum)
        Q4<CT> q;
        q.v[0] = q.v[1] = q.v[2] = q.v[3] = CT(0);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const CT sg = (l < NDIR) ? CT(1) : CT(-1);
            q.v[0] += CT(r[l][0]);
            q.v[1] += sg * CT(r[l][1]);
            q.v[2] += sg * CT(r[l][2]);
            q.v[3] += sg * CT(r[l][3]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) q.v[k] *= CT(2);
        if constexpr (UPD == gfs::UPD_HEATBATH)
            g = to_T<CT>(landau_heatbath(to_d(q), a.T, rng));
        else
            g = finish<UPD, CT>(landau_relax(q), a, rng);
    } else {
        CT D = CT(0), E = CT(0), F = CT(0);
#pragma unroll
        for (int l = 0; l < NL; ++l) su2_mag_add(q_from<CT>(r[l]), l < NDIR, D, E, F);
        if constexpr (UPD == gfs::UPD_HEATBATH) {
            double uu[4];
            rng.draw(0, 0, uu);
            g = to_T<CT>(mag_heatbath(double(D), double(E), double(F), a.T, uu[0], uu[1]));
        } else {
            g = finish<UPD, CT>(mag_relax(D, E, F), a, rng);
        }
    }

    // ---- Step 2: U(x) <- g U(x), U(x - mu) <- U(x - mu) g^dag
    typedef typename std::conditional<ST == gfs::ST_SU2_F32, double, CT>::type AT;
    Q4<AT> ga = q_from<AT>(g.v);
    if constexpr (!std::is_same<AT, CT>::value) q_normalise(ga);
    const Q4<AT> gd = q_dag(ga);
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const bool fw = l < NDIR;
        const int mu = MU0 + (fw ? l : l - NDIR);
        const Q4<AT> m = q_from<AT>(r[l]);
        const Q4<AT> o = fw ? qmul(ga, m) : qmul(m, gd);
#pragma unroll
        for (int k = 0; k < 4; ++k) r[l][k] = S(o.v[k]);
        if (valid) SD::store(plane_ptr<ST>(a.ws, I, fw ? p : 1 - p, mu), I.Vh, lh[l], r[l]);
    }

    // ---- Coulomb: G(x) <- g G(x)
    if constexpr (GAUGE == gfs::COULOMB) {
        V *gp = gacc_ptr<ST>(a.ws, I, p);
        S gr[4];
        SD::load(gp, I.Vh, h, gr);
        const Q4<AT> o = qmul(ga, q_from<AT>(gr));
#pragma unroll
        for (int k = 0; k < 4; ++k) gr[k] = S(o.v[k]);
        if (valid) SD::store(gp, I.Vh, h, gr);
    }
}

// ---------------------------------------------------------------- measures
// the 2x2 complex matrix of a Cayley-Klein 4-vector
__device__ __forceinline__ void ck_matrix(const Q4<double> &u, cx<double> m[2][2]) {
    m[0][0] = cmk(u.v[0], u.v[3]);
    m[0][1] = cmk(u.v[2], u.v[1]);
    m[1][0] = cmk(-u.v[2], u.v[1]);
    m[1][1] = cmk(u.v[0], -u.v[3]);
}

// Per site (tile layout as in the SU(3) measure): F contribution of the
// forward links (Landau/Coulomb Re tr U = 2 u0; MAG |U_00|^2 + |U_11|^2),
// theta of the site (Landau/Coulomb tr Delta Delta^dag with Delta = d.sigma,
// d = sum_mu u_vec(x) - u_vec(x - mu), so 2 |d|^2; MAG |X_01|^2 with
// X = sum_mu U sigma_3 U^dag + U'^dag sigma_3 U', Sec. 2.1.2), and |1 - det U|.
template <int GAUGE, int ST>
__global__ __launch_bounds__(MBLOCK) void k_measure_su2(gfs::MeasureArgs a, const int32_t *active) {
    typedef Store<ST> SD;
    constexpr int NDIR = (GAUGE == gfs::COULOMB) ? 3 : 4;
    constexpr int MU0 = (GAUGE == gfs::COULOMB) ? 1 : 0;
    static_assert(gfs::MTILE_SITES * 2 == MBLOCK, "a measure block covers its tile in both parities");
    __shared__ double sh[4];
    const int tix = xcd_tile(blockIdx.x, gridDim.x);
    const gfs::MTile tl = a.tiles[tix];
    if (active && !active[tl.unit]) return;  // a stopped unit keeps its partial sums
    const gfs::UnitDev U = a.unit[tl.unit];
    const gfs::InstDev I = a.inst[U.inst];
    int32_t j = tl.j0 + (int32_t)(threadIdx.x % gfs::MTILE_SITES);
    const bool valid = j < U.n;
    if (!valid) j = U.n - 1;
    const int32_t h = U.h0 + j;
    const int p = (int)(threadIdx.x / gfs::MTILE_SITES);
    const Site s = site_of(I, h, p);

    double F = 0.0, th = 0.0, us = 0.0, um = 0.0;
    double d[3] = {0.0, 0.0, 0.0};
    cx<double> x01 = cmk(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < NDIR; ++q) {
        const int mu = MU0 + q;
        typename SD::S r[4];
        SD::load(plane_ptr<ST>(a.ws, I, p, mu), I.Vh, h, r);
        const Q4<double> uf = q_from<double>(r);
        SD::load(plane_ptr<ST>(a.ws, I, 1 - p, mu), I.Vh, back_h(I, s, h, mu), r);
        const Q4<double> ub = q_from<double>(r);
        if constexpr (GAUGE == gfs::MAG) {
            F += 2.0 * (uf.v[0] * uf.v[0] + uf.v[3] * uf.v[3]);
            cx<double> m[2][2], n[2][2];
            ck_matrix(uf, m);
            ck_matrix(ub, n);
            // (U s3 U^dag)_01 = U_00 conj(U_10) - U_01 conj(U_11)
            x01 = cadd(x01, csub(cmulc(m[0][0], m[1][0]), cmulc(m[0][1], m[1][1])));
            // (U'^dag s3 U')_01 = conj(U'_00) U'_01 - conj(U'_10) U'_11
            x01 = cadd(x01, csub(cmul(cconj(n[0][0]), n[0][1]), cmul(cconj(n[1][0]), n[1][1])));
        } else {
            F += 2.0 * uf.v[0];
#pragma unroll
            for (int k = 0; k < 3; ++k) d[k] += uf.v[k + 1] - ub.v[k + 1];
        }
    }
    if constexpr (GAUGE == gfs::MAG)
        th = cnorm2(x01);
    else
        th = 2.0 * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (a.with_unitarity) {
        for (int mu = 0; mu < 4; ++mu) {
            typename SD::S r[4];
            SD::load(plane_ptr<ST>(a.ws, I, p, mu), I.Vh, h, r);
            const Q4<double> uf = q_from<double>(r);
            const double e =
                fabs(1.0 - (uf.v[0] * uf.v[0] + uf.v[1] * uf.v[1] + uf.v[2] * uf.v[2] + uf.v[3] * uf.v[3]));
            us += e;
            um = fmax(um, e);
        }
    }
    if (!valid) F = th = us = um = 0.0;
    const double bF = block_sum(F, sh);
    const double bT = block_sum(th, sh);
    double bU = 0.0, bM = 0.0;
    if (a.with_unitarity) {
        bU = block_sum(us, sh);
        bM = block_max(um, sh);
    }
    if (threadIdx.x == 0) {
        double *o = a.partial + 4 * (int64_t)tix;
        o[0] = bF;
        o[1] = bT;
        o[2] = bU;
        o[3] = bM;
    }
}

// ---------------------------------------------------------------- reprojection
// normalise the 4-vector of every (plane, half-site) of the region; stopped
// units are left as they are
template <int ST>
__global__ __launch_bounds__(MBLOCK) void k_reunit_su2(char *ws, int64_t off, int32_t nplanes, int32_t Vp,
                                                        int32_t h_lo, int32_t nh, const int32_t *active,
                                                        int32_t unit0, int32_t hper) {
    typedef Store<ST> SD;
    const int64_t idx = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
    if (idx >= (int64_t)nplanes * nh) return;
    const int32_t pl = (int32_t)(idx / nh), h = h_lo + (int32_t)(idx - (int64_t)pl * nh);
    if (active && !active[unit0 + h / hper]) return;
    typename SD::V *base = reinterpret_cast<typename SD::V *>(ws + off) + (int64_t)pl * SD::NCH * Vp;
    typename SD::S r[4];
    SD::load(base, 0, h, r);
    Q4<double> q = q_from<double>(r);
    q_normalise(q);
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = (typename SD::S)q.v[k];
    SD::store(base, 0, h, r);
}

template <int ST>
__global__ __launch_bounds__(MBLOCK) void k_set_identity_su2(char *ws, int64_t off, int32_t Vh, int32_t Vp) {
    typedef Store<ST> SD;
    const int64_t idx = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
    if (idx >= 2 * (int64_t)Vh) return;
    const int32_t pl = (int32_t)(idx / Vh), h = (int32_t)(idx - (int64_t)pl * Vh);
    typename SD::V *base = reinterpret_cast<typename SD::V *>(ws + off) + (int64_t)pl * SD::NCH * Vp;
    const typename SD::S r[4] = {1, 0, 0, 0};
    SD::store(base, Vh, h, r);
}

// ---------------------------------------------------------------- layout conversion
// natural links (2x2 complex, 8 reals: src[(s - s0) * 32 + mu * 8 + ...]);
// the stored components come from the first row
__device__ __forceinline__ void natural_site(const gfs::InstDev &I, int64_t site, int &p) {
    int64_t r = site;
    const int z = (int)(r % I.n[3]);
    r /= I.n[3];
    const int y = (int)(r % I.n[2]);
    r /= I.n[2];
    const int x = (int)(r % I.n[1]);
    const int t = (int)(r / I.n[1]);
    p = (t + x + y + z) & 1;
}

template <int ST>
__global__ __launch_bounds__(MBLOCK) void k_convert_in_su2(char *ws, gfs::InstDev I, const double *src, int64_t s0,
                                                            int64_t ns) {
    typedef Store<ST> SD;
    const int64_t idx = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
    if (idx >= ns * 4) return;
    const int64_t k = idx >> 2;
    const int mu = (int)(idx & 3);
    int p;
    natural_site(I, s0 + k, p);
    const double *m = src + k * 32 + mu * 8;
    typename SD::S r[4];
    r[0] = (typename SD::S)m[0];  // Re U_00
    r[1] = (typename SD::S)m[3];  // Im U_01
    r[2] = (typename SD::S)m[2];  // Re U_01
    r[3] = (typename SD::S)m[1];  // Im U_00
    SD::store(plane_ptr<ST>(ws, I, p, mu), I.Vh, (int32_t)((s0 + k) >> 1), r);
}

template <int ST>
__global__ __launch_bounds__(MBLOCK) void k_convert_out_su2(const char *ws, gfs::InstDev I, double *dst, int64_t s0,
                                                             int64_t ns, int reunit) {
    typedef Store<ST> SD;
    const int64_t idx = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
    if (idx >= ns * 4) return;
    const int64_t k = idx >> 2;
    const int mu = (int)(idx & 3);
    int p;
    natural_site(I, s0 + k, p);
    typename SD::S r[4];
    SD::load(plane_ptr<ST>(const_cast<char *>(ws), I, p, mu), I.Vh, (int32_t)((s0 + k) >> 1), r);
    Q4<double> q = q_from<double>(r);
    if (reunit) q_normalise(q);
    cx<double> m[2][2];
    ck_matrix(q, m);
    double *o = dst + k * 32 + mu * 8;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            o[2 * (2 * i + jj)] = m[i][jj].re;
            o[2 * (2 * i + jj) + 1] = m[i][jj].im;
        }
}

// U_0(x) <- G(x) U_0(x) G(x + 0)^dag (Coulomb, Sec. 5)
template <int ST>
__global__ __launch_bounds__(MBLOCK) void k_coulomb_fix_su2(char *ws, gfs::InstDev I) {
    typedef Store<ST> SD;
    const int64_t idx = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
    if (idx >= 2 * (int64_t)I.Vh) return;
    const int p = (int)(idx / I.Vh);
    const int32_t h = (int32_t)(idx - (int64_t)p * I.Vh);
    const Site s = site_of(I, h, p);
    typename SD::S r[4];
    SD::load(gacc_ptr<ST>(ws, I, p), I.Vh, h, r);
    const Q4<double> gx = q_from<double>(r);
    SD::load(gacc_ptr<ST>(ws, I, 1 - p), I.Vh, fwd_h(I, s, h, 0), r);
    const Q4<double> gy = q_from<double>(r);
    SD::load(plane_ptr<ST>(ws, I, p, 0), I.Vh, h, r);
    const Q4<double> o = qmul(qmul(gx, q_from<double>(r)), q_dag(gy));
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = (typename SD::S)o.v[k];
    SD::store(plane_ptr<ST>(ws, I, p, 0), I.Vh, h, r);
}

}  // namespace gfd

// ---------------------------------------------------------------- launchers
namespace gfl {

using namespace gfd;

constexpr int NSUB2 = NUPD * NCTD * NBLOCK;

template <int G, int ST, int I>
sweep_fn su2_entry() {
    constexpr int upd = I % NUPD;
    constexpr int ctd = (I / NUPD) % NCTD;
    constexpr int bi = I / (NUPD * NCTD);
    if constexpr (su2_built(upd, ST, ctd, 1, block_of(bi), 0)) {
        typedef typename std::conditional<ctd == 1, double, float>::type CT;
        return &k_sweep_su2<G, upd, ST, CT, block_of(bi)>;
    } else {
        return nullptr;
    }
}

template <int G, int ST, int... I>
std::array<sweep_fn, sizeof...(I)> su2_table(std::integer_sequence<int, I...>) {
    return {{su2_entry<G, ST, I>()...}};
}

template <int G, int ST>
sweep_fn su2_lookup(int upd, int ctd, int bi) {
    static const std::array<sweep_fn, NSUB2> t = su2_table<G, ST>(std::make_integer_sequence<int, NSUB2>{});
    return t[(bi * NCTD + ctd) * NUPD + upd];
}

template <int G>
static sweep_fn su2_by_storage(int upd, int st, int ctd, int bi) {
    if (st == gfs::ST_SU2_F64) return su2_lookup<G, gfs::ST_SU2_F64>(upd, ctd, bi);
    if (st == gfs::ST_SU2_F32) return su2_lookup<G, gfs::ST_SU2_F32>(upd, ctd, bi);
    return su2_lookup<G, gfs::ST_SU2_F32_SP>(upd, ctd, bi);
}

sweep_fn sweep_kernel_su2(int gauge, int upd, int st, int ctd, int W, int B, int nt) {
    if (!su2_built(upd, st, ctd, W, B, nt)) return nullptr;
    const int bi = block_index(B);
    if (gauge == gfs::LANDAU) return su2_by_storage<gfs::LANDAU>(upd, st, ctd, bi);
    if (gauge == gfs::COULOMB) return su2_by_storage<gfs::COULOMB>(upd, st, ctd, bi);
    return su2_by_storage<gfs::MAG>(upd, st, ctd, bi);
}

static inline unsigned nblk_su2(int64_t n) { return (unsigned)((n + MBLOCK - 1) / MBLOCK); }

template <int G>
static void measure_su2_g(int st, unsigned ntiles, hipStream_t s, const gfs::MeasureArgs &a, const int32_t *active) {
    if (st == gfs::ST_SU2_F64)
        k_measure_su2<G, gfs::ST_SU2_F64><<<ntiles, MBLOCK, 0, s>>>(a, active);
    else
        k_measure_su2<G, gfs::ST_SU2_F32><<<ntiles, MBLOCK, 0, s>>>(a, active);
}

hipError_t measure_su2(int gauge, int st, unsigned ntiles, hipStream_t s, const gfs::MeasureArgs &a,
                       const int32_t *active) {
    if (ntiles == 0) return hipSuccess;
    if (gauge == gfs::LANDAU)
        measure_su2_g<gfs::LANDAU>(st, ntiles, s, a, active);
    else if (gauge == gfs::COULOMB)
        measure_su2_g<gfs::COULOMB>(st, ntiles, s, a, active);
    else
        measure_su2_g<gfs::MAG>(st, ntiles, s, a, active);
    return hipGetLastError();
}

hipError_t reunit_su2(int st, char *ws, int64_t off, int32_t nplanes, int32_t Vp, int32_t h_lo, int32_t nh,
                      const int32_t *active, int32_t unit0, int32_t hper, hipStream_t s) {
    const int64_t n = (int64_t)nplanes * nh;
    if (st == gfs::ST_SU2_F64)
        k_reunit_su2<gfs::ST_SU2_F64><<<nblk_su2(n), MBLOCK, 0, s>>>(ws, off, nplanes, Vp, h_lo, nh, active, unit0, hper);
    else
        k_reunit_su2<gfs::ST_SU2_F32><<<nblk_su2(n), MBLOCK, 0, s>>>(ws, off, nplanes, Vp, h_lo, nh, active, unit0, hper);
    return hipGetLastError();
}

hipError_t set_identity_su2(int st, char *ws, int64_t off, int32_t Vh, int32_t Vp, hipStream_t s) {
    const int64_t n = 2 * (int64_t)Vh;
    if (st == gfs::ST_SU2_F64)
        k_set_identity_su2<gfs::ST_SU2_F64><<<nblk_su2(n), MBLOCK, 0, s>>>(ws, off, Vh, Vp);
    else
        k_set_identity_su2<gfs::ST_SU2_F32><<<nblk_su2(n), MBLOCK, 0, s>>>(ws, off, Vh, Vp);
    return hipGetLastError();
}

hipError_t convert_in_su2(int st, char *ws, const gfs::InstDev &I, const double *src, int64_t s0, int64_t ns,
                          hipStream_t s) {
    const int64_t n = 4 * ns;
    if (st == gfs::ST_SU2_F64)
        k_convert_in_su2<gfs::ST_SU2_F64><<<nblk_su2(n), MBLOCK, 0, s>>>(ws, I, src, s0, ns);
    else
        k_convert_in_su2<gfs::ST_SU2_F32><<<nblk_su2(n), MBLOCK, 0, s>>>(ws, I, src, s0, ns);
    return hipGetLastError();
}

hipError_t convert_out_su2(int st, const char *ws, const gfs::InstDev &I, double *dst, int64_t s0, int64_t ns,
                           int reunit, hipStream_t s) {
    const int64_t n = 4 * ns;
    if (st == gfs::ST_SU2_F64)
        k_convert_out_su2<gfs::ST_SU2_F64><<<nblk_su2(n), MBLOCK, 0, s>>>(ws, I, dst, s0, ns, reunit);
    else
        k_convert_out_su2<gfs::ST_SU2_F32><<<nblk_su2(n), MBLOCK, 0, s>>>(ws, I, dst, s0, ns, reunit);
    return hipGetLastError();
}

hipError_t coulomb_fix_su2(int st, char *ws, const gfs::InstDev &I, hipStream_t s) {
    const int64_t n = 2 * (int64_t)I.Vh;
    if (st == gfs::ST_SU2_F64)
        k_coulomb_fix_su2<gfs::ST_SU2_F64><<<nblk_su2(n), MBLOCK, 0, s>>>(ws, I);
    else
        k_coulomb_fix_su2<gfs::ST_SU2_F32><<<nblk_su2(n), MBLOCK, 0, s>>>(ws, I);
    return hipGetLastError();
}

}  // namespace gfl
