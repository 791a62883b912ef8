// gf_kernels.hip -- everything besides the half-sweep: F / theta / unitarity
// reductions in FP64 (Sec. 2.1, Sec. 4.5), per-unit stopping decisions,
// reprojection to SU(3), layout conversion to and from the natural order,
// the Coulomb fix-up of the temporal links, and small bookkeeping kernels.
// The launchers hand the SU(2) storages to their kernels in gf_sweep_su2.hip.
#include "gf_device.hpp"
#include "gf_launch.hpp"
#include "gf_reduce.hpp"

#include <algorithm>
#include <mutex>

namespace gfd {

// traceless part of (K - K^dag)/(2i): sum |.|^2
__device__ __forceinline__ double delta_norm2(const M3<double> &K) {
    // A = (K - K^dag)/(2i): A_ij = ((K_ij - conj K_ji)) / (2i)
    cx<double> A[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const cx<double> d = csub(K.e[i][j], cconj(K.e[j][i]));
            A[i][j] = cmk(0.5 * d.im, -0.5 * d.re);  // d / (2i)
        }
    const double tr = (A[0][0].re + A[1][1].re + A[2][2].re) / 3.0;  // trace is real
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> a = A[i][j];
            if (i == j) a.re -= tr;
            s += cnorm2(a);
        }
    return s;
}

__device__ __forceinline__ cx<double> det3(const M3<double> &m) {
    cx<double> a = cmul(m.e[0][0], csub(cmul(m.e[1][1], m.e[2][2]), cmul(m.e[1][2], m.e[2][1])));
    cx<double> b = cmul(m.e[0][1], csub(cmul(m.e[1][0], m.e[2][2]), cmul(m.e[1][2], m.e[2][0])));
    cx<double> c = cmul(m.e[0][2], csub(cmul(m.e[1][0], m.e[2][1]), cmul(m.e[1][1], m.e[2][0])));
    return cadd(csub(a, b), c);
}

// Per site: F contribution of the forward links, theta of the site;
// optional |1 - det U| of the four forward links.  A block covers the
// MTILE_SITES half-sites of its tile in both parities (waves 0-1 parity 0,
// waves 2-3 parity 1) and tiles are spread over the XCDs in contiguous
// ranges: the backward links of the z, y and x directions are then mostly
// forward links that this block or a recent one on the same XCD has just
// brought into L2, and only the t-direction ones come from further away.
// Partials per tile.
template <int GAUGE, int ST>
__global__ __launch_bounds__(MBLOCK) void k_measure(gfs::MeasureArgs a, const int32_t *active) {
    typedef Store<ST> SD;
    constexpr int NDIR = (GAUGE == gfs::COULOMB) ? 3 : 4;
    constexpr int MU0 = (GAUGE == gfs::COULOMB) ? 1 : 0;
    static_assert(gfs::MTILE_SITES * 2 == MBLOCK, "a measure block covers its tile in both parities");
    __shared__ double sh[4];
    const int tix = xcd_tile(blockIdx.x, gridDim.x);
    const gfs::MTile tl = a.tiles[tix];
    // a stopped unit's links have not changed since its last measurement
    // (the whole block belongs to one unit, so it returns as a whole)
    if (active && !active[tl.unit]) return;
    const gfs::UnitDev U = a.unit[tl.unit];
    const gfs::InstDev I = a.inst[U.inst];
    int32_t j = tl.j0 + (int32_t)(threadIdx.x % gfs::MTILE_SITES);
    const bool valid = j < U.n;
    if (!valid) j = U.n - 1;
    const int32_t h = U.h0 + j;
    const int p = (int)(threadIdx.x / gfs::MTILE_SITES);
    const Site s = site_of(I, h, p);

    double F = 0.0, th = 0.0, us = 0.0, um = 0.0;
    M3<double> K;
    m3_zero(K);  // Landau/Coulomb: K; MAG: W
#pragma unroll
    for (int q = 0; q < NDIR; ++q) {
        const int mu = MU0 + q;
        typename SD::S r[SD::NR];
        M3<double> m;
        SD::load(plane_ptr<ST>(a.ws, I, p, mu), I.Vh, h, r);
        expand<ST, double>(r, m);
        if constexpr (GAUGE == gfs::MAG) {
#pragma unroll
            for (int i = 0; i < 3; ++i) F += cnorm2(m.e[i][i]);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) K.e[i][k] = cadd(K.e[i][k], cmulc(m.e[i][k], m.e[k][k]));
        } else {
            F += m.e[0][0].re + m.e[1][1].re + m.e[2][2].re;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) K.e[i][k] = cadd(K.e[i][k], m.e[i][k]);
        }
        SD::load(plane_ptr<ST>(a.ws, I, 1 - p, mu), I.Vh, back_h(I, s, h, mu), r);
        expand<ST, double>(r, m);
        if constexpr (GAUGE == gfs::MAG) {
            // - diag(U')^dag U'
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const cx<double> t = cmul(cconj(m.e[i][i]), m.e[i][k]);
                    K.e[i][k] = csub(K.e[i][k], t);
                }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) K.e[i][k] = cadd(K.e[i][k], cconj(m.e[k][i]));
        }
    }
    if constexpr (GAUGE == gfs::MAG) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = i + 1; k < 3; ++k) th += cnorm2(csub(K.e[i][k], cconj(K.e[k][i])));
    } else {
        th = delta_norm2(K);
    }
    if (a.with_unitarity) {
        // |1 - det U| of the forward links of every direction (temporal ones too)
        for (int mu = 0; mu < 4; ++mu) {
            typename SD::S r[SD::NR];
            M3<double> m;
            SD::load(plane_ptr<ST>(a.ws, I, p, mu), I.Vh, h, r);
            expand<ST, double>(r, m);
            const cx<double> d = det3(m);
            const double e = sqrt((1.0 - d.re) * (1.0 - d.re) + d.im * d.im);
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

// Stopping decision after a measurement (over all units): a unit stops at
// the first check with theta < tol; counts active units, flags non-finite
// values, sets the FP64-tail flag.
__device__ __forceinline__ void decide_units(int nunits, const double *res, int32_t *active, int32_t *fp64, double tol,
                                             double tail, int32_t *status, double *sh) {
    double cnt = 0.0, bad = 0.0, n64 = 0.0;
    for (int u = threadIdx.x; u < nunits; u += MBLOCK) {
        const double F = __hip_atomic_load(res + 4 * u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double th = __hip_atomic_load(res + 4 * u + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool fin = isfinite(F) && isfinite(th);
        if (!fin) bad += 1.0;
        if (active[u] && th < tol) active[u] = 0;
        if (tail > 0.0) fp64[u] = (th < tail || tail >= 1e300) ? 1 : 0;
        cnt += active[u] ? 1.0 : 0.0;
        n64 += (active[u] && fp64[u]) ? 1.0 : 0.0;
    }
    const double c = block_sum(cnt, sh);
    const double b = block_sum(bad, sh);
    const double d = block_sum(n64, sh);
    if (threadIdx.x == 0) {
        status[0] = (int32_t)c;  // active units
        status[1] = (int32_t)b;  // units with a non-finite F or theta
        status[2] = (int32_t)d;  // active units in the FP64 tail
    }
}

// One block per unit: sum the unit's tile partials in a fixed order and
// normalise: F = sum / (N_c NDIR V_u), theta = sum / (N_c V_u).  With `decide`,
// the last block to finish (device-scope fence + counter) also takes the
// stopping decision over all units and resets the counter.
__global__ __launch_bounds__(MBLOCK) void k_finalize(const gfs::UnitDev *units, const double *partial, int ndir,
                                                     int nc, double *out /* 4 per unit */, int nunits, int decide,
                                                     int32_t *active, int32_t *fp64, double tol, double tail,
                                                     int32_t *status, uint32_t *counter) {
    __shared__ double sh[4];
    __shared__ int last;
    const gfs::UnitDev U = units[blockIdx.x];
    double F = 0.0, th = 0.0, us = 0.0, um = 0.0;
    for (int t = U.mtile0 + threadIdx.x; t < U.mtile1; t += MBLOCK) {
        F += partial[4 * (int64_t)t];
        th += partial[4 * (int64_t)t + 1];
        us += partial[4 * (int64_t)t + 2];
        um = fmax(um, partial[4 * (int64_t)t + 3]);
    }
    const double bF = block_sum(F, sh);
    const double bT = block_sum(th, sh);
    const double bU = block_sum(us, sh);
    const double bM = block_max(um, sh);
    if (threadIdx.x == 0) {
        const double V = 2.0 * (double)U.n;
        out[4 * blockIdx.x] = bF / ((double)nc * ndir * V);
        out[4 * blockIdx.x + 1] = bT / ((double)nc * V);
        out[4 * blockIdx.x + 2] = bU / (4.0 * V);
        out[4 * blockIdx.x + 3] = bM;
    }
    if (!decide) return;
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(counter, 1u);
        last = (prev == (uint32_t)nunits - 1u);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    decide_units(nunits, out, active, fp64, tol, tail, status, sh);
    if (threadIdx.x == 0) *counter = 0u;
}

// After a chunk of n sweeps (units stop only at checks, so a unit active now
// took part in all n): count them for the active units and advance the
// random-stream index of every instance with an active unit.
__global__ void k_count_sweep(int ninst, const gfs::InstDev *inst, const int32_t *active, int32_t *sweeps_done,
                              uint64_t *sweep_ix, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    const gfs::InstDev I = inst[i];
    int any = 0;
    for (int u = I.unit0; u < I.unit0 + I.nunits; ++u)
        if (active[u]) {
            sweeps_done[u] += n;
            any = 1;
        }
    if (any) sweep_ix[i] += (uint64_t)n;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- reprojection
// reproject `count` vectors-of-links: every (plane, site) of the given
// storage region [base, base + nplanes planes of Vh sites)
template <int ST>
__global__ __launch_bounds__(MBLOCK) void k_reunit(char *ws, int64_t off, int32_t nplanes, int32_t Vp, int32_t h_lo,
                                                   int32_t nh, const int32_t *active, int32_t unit0, int32_t hper) {
    typedef Store<ST> SD;
    const int64_t idx = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
    if (idx >= (int64_t)nplanes * nh) return;
    const int32_t pl = (int32_t)(idx / nh), h = h_lo + (int32_t)(idx - (int64_t)pl * nh);
    // a stopped unit keeps the links it stopped with
    if (active && !active[unit0 + h / hper]) return;
    typename SD::V *base = reinterpret_cast<typename SD::V *>(ws + off) + (int64_t)pl * SD::NCH * Vp;
    typename SD::S r[SD::NR];
    SD::load(base, 0, h, r);
    M3<double> m;
    expand<ST, double>(r, m);
    reproject(m);
    compress<ST, double>(m, r);
    SD::store(base, 0, h, r);
}

// identity into the Coulomb accumulator (2 parity planes)
template <int ST>
__global__ __launch_bounds__(MBLOCK) void k_set_identity(char *ws, int64_t off, int32_t Vh, int32_t Vp) {
    typedef Store<ST> SD;
    const int64_t idx = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
    if (idx >= 2 * (int64_t)Vh) return;
    const int32_t pl = (int32_t)(idx / Vh), h = (int32_t)(idx - (int64_t)pl * Vh);
    typename SD::V *base = reinterpret_cast<typename SD::V *>(ws + off) + (int64_t)pl * SD::NCH * Vp;
    M3<double> m;
    m3_identity(m);
    typename SD::S r[SD::NR];
    compress<ST, double>(m, r);
    SD::store(base, Vh, h, r);
}

// ---------------------------------------------------------------- layout conversion
// natural FP64-18 links of sites [s0, s0 + ns) (src[(s - s0)*72 + mu*18 + ...])
// into the parity-split storage
template <int ST>
__global__ __launch_bounds__(MBLOCK) void k_convert_in(char *ws, gfs::InstDev I, const double *src, int64_t s0,
                                                       int64_t ns) {
    typedef Store<ST> SD;
    const int64_t idx = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
    if (idx >= ns * 4) return;
    const int64_t k = idx >> 2;
    const int mu = (int)(idx & 3);
    const int64_t site = s0 + k;
    // parity of the natural index
    int64_t r = site;
    const int z = (int)(r % I.n[3]);
    r /= I.n[3];
    const int y = (int)(r % I.n[2]);
    r /= I.n[2];
    const int x = (int)(r % I.n[1]);
    const int t = (int)(r / I.n[1]);
    const int p = (t + x + y + z) & 1;
    const int32_t h = (int32_t)(site >> 1);
    const double *m = src + k * 72 + mu * 18;
    typename SD::S rr[SD::NR];
#pragma unroll
    for (int c = 0; c < SD::NR; ++c) rr[c] = (typename SD::S)m[c];
    SD::store(plane_ptr<ST>(ws, I, p, mu), I.Vh, h, rr);
}

template <int ST>
__global__ __launch_bounds__(MBLOCK) void k_convert_out(const char *ws, gfs::InstDev I, double *dst, int64_t s0,
                                                        int64_t ns, int reunit) {
    typedef Store<ST> SD;
    const int64_t idx = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
    if (idx >= ns * 4) return;
    const int64_t k = idx >> 2;
    const int mu = (int)(idx & 3);
    const int64_t site = s0 + k;
    int64_t r = site;
    const int z = (int)(r % I.n[3]);
    r /= I.n[3];
    const int y = (int)(r % I.n[2]);
    r /= I.n[2];
    const int x = (int)(r % I.n[1]);
    const int t = (int)(r / I.n[1]);
    const int p = (t + x + y + z) & 1;
    const int32_t h = (int32_t)(site >> 1);
    typename SD::S rr[SD::NR];
    SD::load(plane_ptr<ST>(const_cast<char *>(ws), I, p, mu), I.Vh, h, rr);
    M3<double> m;
    expand<ST, double>(rr, m);
    if (reunit) reproject(m);
    double *o = dst + k * 72 + mu * 18;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            o[2 * (3 * i + jj)] = m.e[i][jj].re;
            o[2 * (3 * i + jj) + 1] = m.e[i][jj].im;
        }
}

// ---------------------------------------------------------------- Coulomb
// U_0(x) <- G(x) U_0(x) G(x + 0)^dag for every site (the accumulated
// transformation of each time-slice applied to the temporal links, Sec. 5)
template <int ST>
__global__ __launch_bounds__(MBLOCK) void k_coulomb_fix(char *ws, gfs::InstDev I) {
    typedef Store<ST> SD;
    const int64_t idx = (int64_t)blockIdx.x * MBLOCK + threadIdx.x;
    if (idx >= 2 * (int64_t)I.Vh) return;
    const int p = (int)(idx / I.Vh);
    const int32_t h = (int32_t)(idx - (int64_t)p * I.Vh);
    const Site s = site_of(I, h, p);
    typename SD::S r[SD::NR];
    M3<double> gx, gy, u, t, o;
    SD::load(gacc_ptr<ST>(ws, I, p), I.Vh, h, r);
    expand<ST, double>(r, gx);
    SD::load(gacc_ptr<ST>(ws, I, 1 - p), I.Vh, fwd_h(I, s, h, 0), r);
    expand<ST, double>(r, gy);
    SD::load(plane_ptr<ST>(ws, I, p, 0), I.Vh, h, r);
    expand<ST, double>(r, u);
    apply_left3(gx, u, t);
    apply_right_dag3(gy, t, o);
    compress<ST, double>(o, r);
    SD::store(plane_ptr<ST>(ws, I, p, 0), I.Vh, h, r);
}


// ---------------------------------------------------------------- no allocation
// F and theta (Sec. 2.1) of an SU(3) field that the caller holds in the
// natural order (18 doubles per link, z fastest, mu = 0 the time direction),
// for callers that cannot allocate: the per-block partial sums go to the
// fixed array `scratch` instead of a workspace.  NA_BLOCKS blocks stride
// over the sites; block b writes partials 2b, 2b+1 on every call, so nothing
// has to start at zero.
constexpr int NA_BLOCKS = 1024;
static __device__ __align__(256) double scratch[2 * NA_BLOCKS];

__device__ __forceinline__ void load_nat(const double *p, M3<double> &m) {
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 v = q[k];
        m.e[k / 3][k % 3] = cmk(v.x, v.y);
    }
}

template <int GAUGE>
__global__ __launch_bounds__(MBLOCK) void k_measure_nat(const double *links, int32_t n0, int32_t n1, int32_t n2,
                                                         int32_t n3, int64_t V, double *part) {
    constexpr int MU0 = (GAUGE == gfs::COULOMB) ? 1 : 0;
    __shared__ double sh[4];
    const int32_t n[4] = {n0, n1, n2, n3};
    // natural-index stride of a step in direction mu
    const int64_t stride[4] = {(int64_t)n1 * n2 * n3, (int64_t)n2 * n3, (int64_t)n3, 1};
    double F = 0.0, th = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * MBLOCK + threadIdx.x; i < V; i += (int64_t)gridDim.x * MBLOCK) {
        M3<double> K;
        m3_zero(K);  // Landau/Coulomb: K; MAG: W
#pragma unroll
        for (int mu = MU0; mu < 4; ++mu) {
            M3<double> m;
            load_nat(links + (i * 4 + mu) * 18, m);
            if constexpr (GAUGE == gfs::MAG) {
#pragma unroll
                for (int a = 0; a < 3; ++a) F += cnorm2(m.e[a][a]);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) K.e[a][b] = cadd(K.e[a][b], cmulc(m.e[a][b], m.e[b][b]));
            } else {
                F += m.e[0][0].re + m.e[1][1].re + m.e[2][2].re;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) K.e[a][b] = cadd(K.e[a][b], m.e[a][b]);
            }
            // x - mu with periodic wrap
            const int32_t c = (int32_t)((i / stride[mu]) % n[mu]);
            const int64_t j = (c == 0) ? i + (int64_t)(n[mu] - 1) * stride[mu] : i - stride[mu];
            load_nat(links + (j * 4 + mu) * 18, m);
            if constexpr (GAUGE == gfs::MAG) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) K.e[a][b] = csub(K.e[a][b], cmul(cconj(m.e[a][a]), m.e[a][b]));
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) K.e[a][b] = cadd(K.e[a][b], cconj(m.e[b][a]));
            }
        }
        if constexpr (GAUGE == gfs::MAG) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = a + 1; b < 3; ++b) th += cnorm2(csub(K.e[a][b], cconj(K.e[b][a])));
        } else {
            th += delta_norm2(K);
        }
    }
    const double bF = block_sum(F, sh);
    const double bT = block_sum(th, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = bF;
        part[2 * blockIdx.x + 1] = bT;
    }
}

// one block: the nb partials in a fixed order, normalised like k_finalize
__global__ __launch_bounds__(MBLOCK) void k_measure_nat_sum(const double *part, int nb, double fnorm, double tnorm,
                                                             double *out) {
    __shared__ double sh[4];
    double F = 0.0, th = 0.0;
    for (int b = threadIdx.x; b < nb; b += MBLOCK) {
        F += part[2 * b];
        th += part[2 * b + 1];
    }
    const double bF = block_sum(F, sh);
    const double bT = block_sum(th, sh);
    if (threadIdx.x == 0) {
        out[0] = bF / fnorm;
        out[1] = bT / tnorm;
    }
}

}  // namespace gfd

// ---------------------------------------------------------------- launchers
namespace gfl {

using namespace gfd;

static inline unsigned nblk(int64_t n) { return (unsigned)((n + MBLOCK - 1) / MBLOCK); }

template <int G>
static hipError_t measure_g(int st, unsigned ntiles, hipStream_t s, const gfs::MeasureArgs &a,
                            const int32_t *active) {
    if (st == gfs::ST_F64R18)
        k_measure<G, gfs::ST_F64R18><<<ntiles, MBLOCK, 0, s>>>(a, active);
    else if (st == gfs::ST_F64R12)
        k_measure<G, gfs::ST_F64R12><<<ntiles, MBLOCK, 0, s>>>(a, active);
    else
        k_measure<G, gfs::ST_F32R12><<<ntiles, MBLOCK, 0, s>>>(a, active);
    return hipGetLastError();
}

hipError_t measure(int gauge, int st, unsigned ntiles, hipStream_t s, const gfs::MeasureArgs &a,
                   const int32_t *active) {
    if (ntiles == 0) return hipSuccess;
    if (gfs::is_su2(st)) return measure_su2(gauge, st, ntiles, s, a, active);
    if (gauge == gfs::LANDAU) return measure_g<gfs::LANDAU>(st, ntiles, s, a, active);
    if (gauge == gfs::COULOMB) return measure_g<gfs::COULOMB>(st, ntiles, s, a, active);
    return measure_g<gfs::MAG>(st, ntiles, s, a, active);
}

hipError_t finalize(int nunits, const gfs::UnitDev *units, const double *partial, int ndir, int nc, double *out,
                    hipStream_t s) {
    k_finalize<<<nunits, MBLOCK, 0, s>>>(units, partial, ndir, nc, out, nunits, 0, nullptr, nullptr, 0.0, 0.0, nullptr,
                                         nullptr);
    return hipGetLastError();
}

hipError_t finalize_decide(int nunits, const gfs::UnitDev *units, const double *partial, int ndir, int nc,
                           double *out, int32_t *active, int32_t *fp64, double tol, double tail, int32_t *status,
                           uint32_t *counter, hipStream_t s) {
    k_finalize<<<nunits, MBLOCK, 0, s>>>(units, partial, ndir, nc, out, nunits, 1, active, fp64, tol, tail, status,
                                         counter);
    return hipGetLastError();
}

hipError_t count_sweep(int ninst, const gfs::InstDev *inst, const int32_t *active, int32_t *sweeps_done,
                       uint64_t *sweep_ix, int32_t n, hipStream_t s) {
    k_count_sweep<<<(ninst + 63) / 64, 64, 0, s>>>(ninst, inst, active, sweeps_done, sweep_ix, n);
    return hipGetLastError();
}

hipError_t fill_i32(int32_t *p, int32_t v, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<(n + 255) / 256, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t reunit(int st, char *ws, int64_t off, int32_t nplanes, int32_t Vh, int32_t Vp, int32_t h_lo, int32_t nh,
                  const int32_t *active, int32_t unit0, int32_t nunits, hipStream_t s) {
    const int64_t n = (int64_t)nplanes * nh;
    if (n <= 0) return hipSuccess;
    const int32_t hper = Vh / nunits;
    if (gfs::is_su2(st)) return reunit_su2(st, ws, off, nplanes, Vp, h_lo, nh, active, unit0, hper, s);
    if (st == gfs::ST_F64R18)
        k_reunit<gfs::ST_F64R18><<<nblk(n), MBLOCK, 0, s>>>(ws, off, nplanes, Vp, h_lo, nh, active, unit0, hper);
    else if (st == gfs::ST_F64R12)
        k_reunit<gfs::ST_F64R12><<<nblk(n), MBLOCK, 0, s>>>(ws, off, nplanes, Vp, h_lo, nh, active, unit0, hper);
    else
        k_reunit<gfs::ST_F32R12><<<nblk(n), MBLOCK, 0, s>>>(ws, off, nplanes, Vp, h_lo, nh, active, unit0, hper);
    return hipGetLastError();
}

hipError_t set_identity(int st, char *ws, int64_t off, int32_t Vh, int32_t Vp, hipStream_t s) {
    if (gfs::is_su2(st)) return set_identity_su2(st, ws, off, Vh, Vp, s);
    const int64_t n = 2 * (int64_t)Vh;
    if (st == gfs::ST_F64R18)
        k_set_identity<gfs::ST_F64R18><<<nblk(n), MBLOCK, 0, s>>>(ws, off, Vh, Vp);
    else if (st == gfs::ST_F64R12)
        k_set_identity<gfs::ST_F64R12><<<nblk(n), MBLOCK, 0, s>>>(ws, off, Vh, Vp);
    else
        k_set_identity<gfs::ST_F32R12><<<nblk(n), MBLOCK, 0, s>>>(ws, off, Vh, Vp);
    return hipGetLastError();
}

hipError_t convert_in(int st, char *ws, const gfs::InstDev &I, const double *src, int64_t s0, int64_t ns,
                      hipStream_t s) {
    if (gfs::is_su2(st)) return convert_in_su2(st, ws, I, src, s0, ns, s);
    const int64_t n = 4 * ns;
    if (st == gfs::ST_F64R18)
        k_convert_in<gfs::ST_F64R18><<<nblk(n), MBLOCK, 0, s>>>(ws, I, src, s0, ns);
    else if (st == gfs::ST_F64R12)
        k_convert_in<gfs::ST_F64R12><<<nblk(n), MBLOCK, 0, s>>>(ws, I, src, s0, ns);
    else
        k_convert_in<gfs::ST_F32R12><<<nblk(n), MBLOCK, 0, s>>>(ws, I, src, s0, ns);
    return hipGetLastError();
}

hipError_t convert_out(int st, const char *ws, const gfs::InstDev &I, double *dst, int64_t s0, int64_t ns, int reunit,
                       hipStream_t s) {
    if (gfs::is_su2(st)) return convert_out_su2(st, ws, I, dst, s0, ns, reunit, s);
    const int64_t n = 4 * ns;
    if (st == gfs::ST_F64R18)
        k_convert_out<gfs::ST_F64R18><<<nblk(n), MBLOCK, 0, s>>>(ws, I, dst, s0, ns, reunit);
    else if (st == gfs::ST_F64R12)
        k_convert_out<gfs::ST_F64R12><<<nblk(n), MBLOCK, 0, s>>>(ws, I, dst, s0, ns, reunit);
    else
        k_convert_out<gfs::ST_F32R12><<<nblk(n), MBLOCK, 0, s>>>(ws, I, dst, s0, ns, reunit);
    return hipGetLastError();
}

hipError_t coulomb_fix(int st, char *ws, const gfs::InstDev &I, hipStream_t s) {
    if (gfs::is_su2(st)) return coulomb_fix_su2(st, ws, I, s);
    const int64_t n = 2 * (int64_t)I.Vh;
    if (st == gfs::ST_F64R18)
        k_coulomb_fix<gfs::ST_F64R18><<<nblk(n), MBLOCK, 0, s>>>(ws, I);
    else if (st == gfs::ST_F64R12)
        k_coulomb_fix<gfs::ST_F64R12><<<nblk(n), MBLOCK, 0, s>>>(ws, I);
    else
        k_coulomb_fix<gfs::ST_F32R12><<<nblk(n), MBLOCK, 0, s>>>(ws, I);
    return hipGetLastError();
}


// Address of this device's copy of `scratch`, looked up once per device with
// that device current (each device holds its own copy at its own address;
// the array's name is only a host-side stand-in).
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[64] = {};

hipError_t noalloc_scratch(int dev, double **ptr, size_t *bytes) {
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *ptr = g_scratch_ptr[dev];
    if (bytes) *bytes = sizeof(scratch);
    return hipSuccess;
}

hipError_t measure_nat(int gauge, const double *links, const int32_t n[4], double *out, double *scr, hipStream_t s) {
    const int64_t V = (int64_t)n[0] * n[1] * n[2] * n[3];
    const int nb = (int)std::min<int64_t>(NA_BLOCKS, (V + MBLOCK - 1) / MBLOCK);
    const int ndir = (gauge == gfs::COULOMB) ? 3 : 4;
    if (gauge == gfs::LANDAU)
        k_measure_nat<gfs::LANDAU><<<nb, MBLOCK, 0, s>>>(links, n[0], n[1], n[2], n[3], V, scr);
    else if (gauge == gfs::COULOMB)
        k_measure_nat<gfs::COULOMB><<<nb, MBLOCK, 0, s>>>(links, n[0], n[1], n[2], n[3], V, scr);
    else
        k_measure_nat<gfs::MAG><<<nb, MBLOCK, 0, s>>>(links, n[0], n[1], n[2], n[3], V, scr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_measure_nat_sum<<<1, MBLOCK, 0, s>>>(scr, nb, 3.0 * ndir * (double)V, 3.0 * (double)V, out);
    return hipGetLastError();
}

}  // namespace gfl
