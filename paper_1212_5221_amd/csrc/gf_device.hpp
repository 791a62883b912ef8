// gf_device.hpp -- device-side building blocks of libgf for gfx950:
// complex/SU(3) arithmetic in registers, the parity-split structure-of-arrays
// link storage, lattice indexing on half-site indices, and Philox4x64-10.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf_shared.hpp"

namespace gfd {

// ---------------------------------------------------------------- complex
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cmk(T r, T i) {
    cx<T> c;
    c.re = r;
    c.im = i;
    return c;
}
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) {
    return cmk(a.re + b.re, a.im + b.im);
}
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) {
    return cmk(a.re - b.re, a.im - b.im);
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) {
    return cmk(a.re, -a.im);
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return cmk(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
// acc + a*b
template <typename T>
__device__ __forceinline__ cx<T> cmac(cx<T> acc, cx<T> a, cx<T> b) {
    return cmk(acc.re + a.re * b.re - a.im * b.im, acc.im + a.re * b.im + a.im * b.re);
}
// acc + a*conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmacc(cx<T> acc, cx<T> a, cx<T> b) {
    return cmk(acc.re + a.re * b.re + a.im * b.im, acc.im + a.im * b.re - a.re * b.im);
}
template <typename T>
__device__ __forceinline__ T cnorm2(cx<T> a) {
    return a.re * a.re + a.im * a.im;
}

// 3x3 complex matrix in registers
template <typename T>
struct M3 {
    cx<T> e[3][3];
};

template <typename T>
__device__ __forceinline__ void m3_identity(M3<T> &m) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) m.e[i][j] = cmk<T>(i == j ? T(1) : T(0), T(0));
}

template <typename T>
__device__ __forceinline__ void m3_zero(M3<T> &m) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) m.e[i][j] = cmk<T>(T(0), T(0));
}

// third row of an SU(3) matrix from the first two: (u x v)^*  (Sec. 4.2)
template <typename T>
__device__ __forceinline__ void m3_row2(M3<T> &m) {
    const cx<T> *u = m.e[0], *v = m.e[1];
    m.e[2][0] = cconj(csub(cmul(u[1], v[2]), cmul(u[2], v[1])));
    m.e[2][1] = cconj(csub(cmul(u[2], v[0]), cmul(u[0], v[2])));
    m.e[2][2] = cconj(csub(cmul(u[0], v[1]), cmul(u[1], v[0])));
}

// out = a b
template <typename T>
__device__ __forceinline__ void apply_left3(const M3<T> &a, const M3<T> &b, M3<T> &out) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmul(a.e[i][0], b.e[0][j]);
            s = cmac(s, a.e[i][1], b.e[1][j]);
            out.e[i][j] = cmac(s, a.e[i][2], b.e[2][j]);
        }
}

// out = b a^dag
template <typename T>
__device__ __forceinline__ void apply_right_dag3(const M3<T> &a, const M3<T> &b, M3<T> &out) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmulc(b.e[i][0], a.e[j][0]);
            s = cmacc(s, b.e[i][1], a.e[j][1]);
            out.e[i][j] = cmacc(s, b.e[i][2], a.e[j][2]);
        }
}

// reprojection to SU(3) (Sec. 4.5): normalise row 0, Gram-Schmidt row 1,
// row 2 = (row0 x row1)^*
template <typename T>
__device__ __forceinline__ void reproject(M3<T> &m) {
    const T n0 = T(1) / sqrt(cnorm2(m.e[0][0]) + cnorm2(m.e[0][1]) + cnorm2(m.e[0][2]));
#pragma unroll
    for (int k = 0; k < 3; ++k) m.e[0][k] = cmk(m.e[0][k].re * n0, m.e[0][k].im * n0);
    cx<T> pr = cmk(T(0), T(0));
#pragma unroll
    for (int k = 0; k < 3; ++k) pr = cadd(pr, cmulc(m.e[1][k], m.e[0][k]));  // conj(row0) . row1
#pragma unroll
    for (int k = 0; k < 3; ++k) m.e[1][k] = csub(m.e[1][k], cmul(pr, m.e[0][k]));
    const T n1 = T(1) / sqrt(cnorm2(m.e[1][0]) + cnorm2(m.e[1][1]) + cnorm2(m.e[1][2]));
#pragma unroll
    for (int k = 0; k < 3; ++k) m.e[1][k] = cmk(m.e[1][k].re * n1, m.e[1][k].im * n1);
    m3_row2(m);
}

// One first-order renormalisation of the two stored rows of a 12-real link:
// each row r <- r (3 - |r|^2) / 2, which takes a norm 1 + d to 1 + O(d^2)
// with no division or square root.  The rebuilt third row scales with the
// product of the two row norms, so under left multiplication by unitary
// matrices far from the identity a norm defect of the stored rows grows by
// about 4/3 per update, and links that keep receiving large updates
// (annealing, the first sweeps from a random gauge) would leave SU(3)
// exponentially fast.  Right multiplication by a unitary matrix keeps the
// norms and the overlap of the stored rows and needs no correction; the
// overlap does not grow under left multiplication either (checked in a
// model with random SU(3) updates, where norm correction alone keeps the
// defect at the storage rounding over 10^4 updates).
template <typename T>
__device__ __forceinline__ void renormalise_rows(M3<T> &m) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const T s = T(1.5) - T(0.5) * (cnorm2(m.e[i][0]) + cnorm2(m.e[i][1]) + cnorm2(m.e[i][2]));
#pragma unroll
        for (int k = 0; k < 3; ++k) m.e[i][k] = cmk(m.e[i][k].re * s, m.e[i][k].im * s);
    }
}

// SU(2) element as 4 reals (g0, g1, g2, g3): [[g0 + i g3, g2 + i g1], [-g2 + i g1, g0 - i g3]]
template <typename T>
struct Q4 {
    T v[4];
};

// rows i,j of M <- g rows i,j
template <typename T>
__device__ __forceinline__ void left_sub(M3<T> &m, int i, int j, const Q4<T> &g) {
    const cx<T> a = cmk(g.v[0], g.v[3]), b = cmk(g.v[2], g.v[1]), c = cmk(-g.v[2], g.v[1]), d = cmk(g.v[0], -g.v[3]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        cx<T> mi = m.e[i][k], mj = m.e[j][k];
        m.e[i][k] = cmac(cmul(a, mi), b, mj);
        m.e[j][k] = cmac(cmul(c, mi), d, mj);
    }
}

template <typename T>
__device__ __forceinline__ Q4<T> qmul(const Q4<T> &a, const Q4<T> &b) {
    // product of the 2x2 Cayley-Klein matrices
    Q4<T> r;
    r.v[0] = a.v[0] * b.v[0] - a.v[1] * b.v[1] - a.v[2] * b.v[2] - a.v[3] * b.v[3];
    r.v[1] = a.v[0] * b.v[1] + a.v[1] * b.v[0] - a.v[2] * b.v[3] + a.v[3] * b.v[2];
    r.v[2] = a.v[0] * b.v[2] + a.v[2] * b.v[0] - a.v[3] * b.v[1] + a.v[1] * b.v[3];
    r.v[3] = a.v[0] * b.v[3] + a.v[3] * b.v[0] - a.v[1] * b.v[2] + a.v[2] * b.v[1];
    return r;
}

// ---------------------------------------------------------------- launch
// Workgroups are dispatched round-robin over the 8 XCDs; block b works on
// tile xcd_tile(b, n), which gives every XCD a contiguous range of tiles so
// that neighbouring tiles share an L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, i = b >> 3;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ---------------------------------------------------------------- storage
// Link storage (per instance, parity-split structure of arrays):
//   plane (p, mu) holds Vp = Vh rounded up to 16 sites of NCH 16-byte
//   vectors each, in blocks of 16 sites (see site_vec).
// F32R12: 3 float4 chunks = rows 0,1 as (re,im) pairs.
// F64R12: 6 double2 chunks = the 6 complex entries of rows 0,1.
// F64R18: 9 double2 chunks = all 9 complex entries.
// Sites are grouped in blocks of 16: chunk c of half-site h is the 16-byte
// vector at base + ((h / 16) NCH + c) 16 + h % 16.  A wavefront of 64
// consecutive sites reads 4 contiguous 256-byte segments per chunk, and one
// address per link serves all chunks (immediate offsets c * 256 bytes).
template <int NCH, typename V>
__device__ __forceinline__ const V *site_vec(const V *base, uint32_t h) {
    return base + (size_t)(h >> 4) * (NCH * 16) + (h & 15u);
}
template <int NCH, typename V>
__device__ __forceinline__ V *site_vec(V *base, uint32_t h) {
    return base + (size_t)(h >> 4) * (NCH * 16) + (h & 15u);
}

// one 16-byte vector access; NT: non-temporal (streaming) cache policy
// (the builtins take native vector types)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ float4 ld16(const float4 *p) {
    if constexpr (NT) {
        const f32x4 n = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
        return make_float4(n.x, n.y, n.z, n.w);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ double2 ld16(const double2 *p) {
    if constexpr (NT) {
        const f64x2 n = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p));
        return make_double2(n.x, n.y);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ void st16(float4 *p, const float4 &v) {
    if constexpr (NT) {
        f32x4 n = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(n, reinterpret_cast<f32x4 *>(p));
    } else {
        *p = v;
    }
}
template <bool NT>
__device__ __forceinline__ void st16(double2 *p, const double2 &v) {
    if constexpr (NT) {
        f64x2 n = {v.x, v.y};
        __builtin_nontemporal_store(n, reinterpret_cast<f64x2 *>(p));
    } else {
        *p = v;
    }
}

template <int ST>
struct Store;

template <>
struct Store<gfs::ST_F32R12> {
    typedef float S;
    typedef float4 V;
    static constexpr int NR = 12, NCH = 3, ROWS = 2;
    template <bool NT = false>
    __device__ static __forceinline__ void load(const V *__restrict__ base, int64_t Vh, int64_t h, S r[NR]) {
        const V *sv = site_vec<NCH>(base, (uint32_t)h);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            V v = ld16<NT>(sv + 16 * c);
            r[4 * c] = v.x;
            r[4 * c + 1] = v.y;
            r[4 * c + 2] = v.z;
            r[4 * c + 3] = v.w;
        }
    }
    template <bool NT = false>
    __device__ static __forceinline__ void store(V *__restrict__ base, int64_t Vh, int64_t h, const S r[NR]) {
        V *sv = site_vec<NCH>(base, (uint32_t)h);
#pragma unroll
        for (int c = 0; c < NCH; ++c) st16<NT>(sv + 16 * c, make_float4(r[4 * c], r[4 * c + 1], r[4 * c + 2], r[4 * c + 3]));
    }
};

template <>
struct Store<gfs::ST_F32R12_SP> : Store<gfs::ST_F32R12> {};

template <>
struct Store<gfs::ST_F64R12> {
    typedef double S;
    typedef double2 V;
    static constexpr int NR = 12, NCH = 6, ROWS = 2;
    template <bool NT = false>
    __device__ static __forceinline__ void load(const V *__restrict__ base, int64_t Vh, int64_t h, S r[NR]) {
        const V *sv = site_vec<NCH>(base, (uint32_t)h);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            V v = ld16<NT>(sv + 16 * c);
            r[2 * c] = v.x;
            r[2 * c + 1] = v.y;
        }
    }
    template <bool NT = false>
    __device__ static __forceinline__ void store(V *__restrict__ base, int64_t Vh, int64_t h, const S r[NR]) {
        V *sv = site_vec<NCH>(base, (uint32_t)h);
#pragma unroll
        for (int c = 0; c < NCH; ++c) st16<NT>(sv + 16 * c, make_double2(r[2 * c], r[2 * c + 1]));
    }
};

template <>
struct Store<gfs::ST_F64R18> {
    typedef double S;
    typedef double2 V;
    static constexpr int NR = 18, NCH = 9, ROWS = 3;
    template <bool NT = false>
    __device__ static __forceinline__ void load(const V *__restrict__ base, int64_t Vh, int64_t h, S r[NR]) {
        const V *sv = site_vec<NCH>(base, (uint32_t)h);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            V v = ld16<NT>(sv + 16 * c);
            r[2 * c] = v.x;
            r[2 * c + 1] = v.y;
        }
    }
    template <bool NT = false>
    __device__ static __forceinline__ void store(V *__restrict__ base, int64_t Vh, int64_t h, const S r[NR]) {
        V *sv = site_vec<NCH>(base, (uint32_t)h);
#pragma unroll
        for (int c = 0; c < NCH; ++c) st16<NT>(sv + 16 * c, make_double2(r[2 * c], r[2 * c + 1]));
    }
};

// registers (storage precision) -> full matrix in compute precision
template <int ST, typename T>
__device__ __forceinline__ void expand(const typename Store<ST>::S *r, M3<T> &m) {
    constexpr int ROWS = Store<ST>::ROWS;
#pragma unroll
    for (int i = 0; i < ROWS; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) m.e[i][j] = cmk<T>(T(r[2 * (3 * i + j)]), T(r[2 * (3 * i + j) + 1]));
    if (ROWS == 2) m3_row2(m);
}

// the stored rows of m back to registers (rounding to the storage precision)
template <int ST, typename T>
__device__ __forceinline__ void compress(const M3<T> &m, typename Store<ST>::S *r) {
    typedef typename Store<ST>::S S;
    constexpr int ROWS = Store<ST>::ROWS;
#pragma unroll
    for (int i = 0; i < ROWS; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            r[2 * (3 * i + j)] = S(m.e[i][j].re);
            r[2 * (3 * i + j) + 1] = S(m.e[i][j].im);
        }
}

template <int ST>
__device__ __forceinline__ typename Store<ST>::V *plane_ptr(char *ws, const gfs::InstDev &I, int p, int mu) {
    typedef typename Store<ST>::V V;
    return reinterpret_cast<V *>(ws + I.links_off) + (int64_t)((p * 4 + mu) * Store<ST>::NCH) * I.Vp;
}

template <int ST>
__device__ __forceinline__ typename Store<ST>::V *gacc_ptr(char *ws, const gfs::InstDev &I, int p) {
    typedef typename Store<ST>::V V;
    return reinterpret_cast<V *>(ws + I.g_off) + (int64_t)(p * Store<ST>::NCH) * I.Vp;
}

// ---------------------------------------------------------------- geometry
// Half-site index h = floor(i/2) of the natural index i = ((t Nx + x) Ny + y) Nz + z
// (Nz even).  The pair h holds one site of each parity; the z-bit b of the
// site of 4D parity p is (p - t - x - y) mod 2.
struct Site {
    int t, x, y, hz, b;
};

__device__ __forceinline__ Site site_of(const gfs::InstDev &I, int32_t h, int p) {
    Site s;
    const int32_t hzn = I.n[3] >> 1;
    int32_t r = h / hzn;
    s.hz = h - r * hzn;
    int32_t r2 = r / I.n[2];
    s.y = r - r2 * I.n[2];
    s.t = r2 / I.n[1];
    s.x = r2 - s.t * I.n[1];
    s.b = (p - s.t - s.x - s.y) & 1;
    return s;
}

// half-index of the backward neighbour x - mu (it has the opposite parity)
__device__ __forceinline__ int32_t back_h(const gfs::InstDev &I, const Site &s, int32_t h, int mu) {
    const int32_t S2 = I.n[3] >> 1, S1 = I.n[2] * S2, S0 = I.n[1] * S1;
    switch (mu) {
    case 0:
        return s.t == 0 ? h + (I.n[0] - 1) * S0 : h - S0;
    case 1:
        return s.x == 0 ? h + (I.n[1] - 1) * S1 : h - S1;
    case 2:
        return s.y == 0 ? h + (I.n[2] - 1) * S2 : h - S2;
    default:
        return s.b ? h : (s.hz == 0 ? h + S2 - 1 : h - 1);
    }
}

// half-index of the forward neighbour x + mu (opposite parity)
__device__ __forceinline__ int32_t fwd_h(const gfs::InstDev &I, const Site &s, int32_t h, int mu) {
    const int32_t S2 = I.n[3] >> 1, S1 = I.n[2] * S2, S0 = I.n[1] * S1;
    switch (mu) {
    case 0:
        return s.t == I.n[0] - 1 ? h - (I.n[0] - 1) * S0 : h + S0;
    case 1:
        return s.x == I.n[1] - 1 ? h - (I.n[1] - 1) * S1 : h + S1;
    case 2:
        return s.y == I.n[2] - 1 ? h - (I.n[2] - 1) * S2 : h + S2;
    default:
        return s.b == 0 ? h : (s.hz == S2 - 1 ? h - S2 + 1 : h + 1);
    }
}

__device__ __forceinline__ int64_t natural_index(const gfs::InstDev &I, const Site &s) {
    return ((((int64_t)s.t * I.n[1] + s.x) * I.n[2] + s.y) * I.n[3]) + 2 * s.hz + s.b;
}

// ---------------------------------------------------------------- Philox4x64-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): 10 rounds of the 4x64 bijection with a Weyl-sequence key schedule.
// The 128-bit product a b as (lo, hi) from four 32 x 32 -> 64 products
// (schoolbook; each partial sum stays below 2^64), so that low and high
// halves share their partial products (one v_mad_u64_u32 each).
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi) {
    const uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32), bl = (uint32_t)b, bh = (uint32_t)(b >> 32);
    const uint64_t p0 = (uint64_t)al * bl;
    const uint64_t p1 = (uint64_t)al * bh + (p0 >> 32);
    const uint64_t p2 = (uint64_t)ah * bl + (uint32_t)p1;
    const uint64_t p3 = (uint64_t)ah * bh + (p1 >> 32) + (p2 >> 32);
    lo = (p2 << 32) | (uint32_t)p0;
    hi = p3;
}

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t lo0, hi0, lo1, hi1;
        mulhilo64(M0, c[0], lo0, hi0);
        mulhilo64(M1, c[2], lo1, hi1);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

__device__ __forceinline__ double unit_open(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1.0p-53; }

struct Rng {
    uint64_t k0, k1, sweep, site, sg;
    __device__ __forceinline__ void draw(uint64_t block, uint64_t stream, double u[4]) const {
        uint64_t c[4] = {sweep, site, (sg << 16) | block, stream};
        philox4x64_10(c, k0, k1);
#pragma unroll
        for (int q = 0; q < 4; ++q) u[q] = unit_open(c[q]);
    }
};

}  // namespace gfd
