// gf_shared.hpp -- plain structs and enums shared by the host library and the
// HIP kernels of libgf (never by the CPU oracle).
#pragma once

#include <stdint.h>

namespace gfs {

enum Gauge { LANDAU = 0, COULOMB = 1, MAG = 2 };
enum Update { UPD_OR = 0, UPD_MICRO = 1, UPD_HEATBATH = 2, UPD_SR = 3 };
// ST_F32R12_SP is the ST_F32R12 storage; its half-sweep kernels also apply G
// in FP32 (single precision throughout, the F/theta sums and reprojection
// aside).  ST_SU2_*: links of the gauge group SU(2) as their 4 Cayley-Klein
// components; ST_SU2_F32_SP is ST_SU2_F32 with g applied in FP32.
enum Storage {
    ST_F64R18 = 0,
    ST_F64R12 = 1,
    ST_F32R12 = 2,
    ST_F32R12_SP = 3,
    ST_SU2_F64 = 4,
    ST_SU2_F32 = 5,
    ST_SU2_F32_SP = 6
};
constexpr bool is_su2(int st) { return st == ST_SU2_F64 || st == ST_SU2_F32 || st == ST_SU2_F32_SP; }

// one lattice instance, as the kernels see it
struct InstDev {
    int32_t n[4];      // Nt, Nx, Ny, Nz
    int32_t Vh;        // half the number of sites
    int32_t unit0;     // first unit of this instance
    int32_t nunits;    // 1 (Landau, MAG) or Nt (Coulomb)
    int32_t Vp;        // Vh rounded up to a multiple of 16 (plane stride in sites)
    int64_t links_off; // byte offset of the link planes in the workspace
    int64_t g_off;     // byte offset of the Coulomb accumulator (or -1)
};

// one independently stopping unit: a whole instance, or one Coulomb time-slice
struct UnitDev {
    int32_t inst;
    int32_t t;       // time-slice (Coulomb) or -1
    int32_t h0;      // first half-site index of the unit
    int32_t n;       // half-sites of the unit (sites of one parity)
    int32_t mtile0;  // measure tiles [mtile0, mtile1) belong to this unit
    int32_t mtile1;
};

// a sweep tile: sites [j0, j0 + sites_per_block) of one unit
struct Tile {
    int32_t unit;
    int32_t j0;
};

// half-sites per measure tile (a 256-thread block covers them in both parities)
constexpr int MTILE_SITES = 128;

// a measure tile: half-sites [j0, j0 + MTILE_SITES) of one unit, both
// parities (parity is unused)
struct MTile {
    int32_t unit;
    int32_t parity;
    int32_t j0;
    int32_t pad;
};

struct SweepArgs {
    char *ws;
    const InstDev *inst;
    const UnitDev *unit;
    const Tile *tiles;
    const int32_t *active;    // per unit
    const int32_t *fp64;      // per unit: tail flag (mixed storage)
    const uint64_t *sweep_ix; // per instance: global sweep index (random counter)
    int32_t parity;           // active parity (Coulomb: 3D parity)
    int32_t fp64_select;      // -1 all units, else only units whose flag equals it
    int32_t sweep_off;        // random counter = sweep_ix[inst] + sweep_off (sweeps counted per chunk)
    int32_t xcd_order;        // 1: block b works on tile xcd_tile(b, n) (contiguous per XCD), 0: on tile b
    double omega, T, p_sr;
    uint64_t seed;
};

struct MeasureArgs {
    char *ws;
    const InstDev *inst;
    const UnitDev *unit;
    const MTile *tiles;
    double *partial; // 4 doubles per measure tile: F, theta, sum |1-det|, max |1-det|
    int32_t with_unitarity;
};

}  // namespace gfs
