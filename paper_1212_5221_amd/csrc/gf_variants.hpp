// gf_variants.hpp -- which half-sweep kernel variants exist, and their place
// in the lookup tables.  A variant is (update, storage, compute precision)
// and a launch shape (wavefronts W per group of 64 sites, threads B per
// block, cached or non-temporal link traffic).  su3_built() and su2_built()
// are the only places that say which variants are built; the tables are
// generated from them (gf_sweep_table.hpp) and the autotuner and the tests
// enumerate the shapes through the same predicate.
#pragma once

#include "gf_shared.hpp"

namespace gfl {

constexpr int NWAVE = 3;   // W = 1, 2, 4
constexpr int NBLOCK = 4;  // B = 64, 128, 256, 512
constexpr int NNT = 2;     // 0: cached loads and stores; 1: non-temporal
constexpr int NUPD = 4;    // gfs::Update
constexpr int NCTD = 2;    // compute precision of the update: 0 FP32, 1 FP64
constexpr int NSUB = NUPD * NCTD * NWAVE * NBLOCK * NNT;  // entries per (gauge, storage)

constexpr int wave_of(int wi) { return 1 << wi; }
constexpr int block_of(int bi) { return 64 << bi; }
// index of W (B) in its dimension, -1 if it is not one of the values
constexpr int wave_index(int W) { return W == 1 ? 0 : W == 2 ? 1 : W == 4 ? 2 : -1; }
constexpr int block_index(int B) { return B == 64 ? 0 : B == 128 ? 1 : B == 256 ? 2 : B == 512 ? 3 : -1; }

constexpr int sub_index(int upd, int ctd, int wi, int bi, int nt) {
    return (((nt * NBLOCK + bi) * NWAVE + wi) * NCTD + ctd) * NUPD + upd;
}

constexpr bool is_random(int upd) { return upd == gfs::UPD_HEATBATH || upd == gfs::UPD_SR; }

// SU(3):
//  - FP64 storage updates in FP64; mixed FP32 storage in FP32 or FP64
//    (stochastic relaxation in FP64 only; the heatbath's local algebra in
//    either, its sample always in FP64);
//    single precision: overrelaxation and microcanonical steps in FP32;
//  - W divides the site's links (8, Coulomb 6) and a block holds at least
//    one group of 64 sites (B >= 64 W);
//  - a 512-thread block leaves a lane 256 registers: not enough for an FP64
//    update with one wavefront per site group (all 8 links of a site in
//    one lane) or for the FP64 random updates, which would spill;
//  - non-temporal variants for the streaming updates (overrelaxation and
//    microcanonical); the random updates are bound by arithmetic.
constexpr bool su3_built(int gauge, int upd, int st, int ctd, int W, int B, int nt) {
    const int nl = gauge == gfs::COULOMB ? 6 : 8;
    if (W < 1 || nl % W != 0 || B < 64 * W) return false;
    if (nt && is_random(upd)) return false;
    if (B == 512 && ctd == 1 && (W == 1 || is_random(upd))) return false;
    if (st == gfs::ST_F64R18 || st == gfs::ST_F64R12) return ctd == 1;
    if (st == gfs::ST_F32R12) return ctd == 1 || upd != gfs::UPD_SR;
    if (st == gfs::ST_F32R12_SP) return ctd == 0 && !is_random(upd);
    return false;
}

// SU(2): one lane per site (W = 1), cached traffic; FP64 storage in FP64;
// mixed FP32 in FP32 or FP64 (random updates FP64); single precision FP32.
constexpr bool su2_built(int upd, int st, int ctd, int W, int B, int nt) {
    if (W != 1 || nt != 0 || block_index(B) < 0) return false;
    if (st == gfs::ST_SU2_F64) return ctd == 1;
    if (st == gfs::ST_SU2_F32) return ctd == 1 || !is_random(upd);
    if (st == gfs::ST_SU2_F32_SP) return ctd == 0 && !is_random(upd);
    return false;
}

}  // namespace gfl
