// gf_launch.hpp -- host-side launchers of the libgf kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf_shared.hpp"

namespace gfl {

// the half-sweep kernel variant for (gauge, update, storage, compute in
// double?) and launch shape (W wavefronts per site group, B threads per
// block, non-temporal link traffic nt); nullptr if not built (the variants
// are those gf_variants.hpp declares built)
typedef void (*sweep_fn)(gfs::SweepArgs);
sweep_fn sweep_kernel(int gauge, int upd, int st, int ct_double, int W, int B, int nt);
// the SU(3) table of one gauge and storage (gf_sweep_table.hpp), indexed by
// the positions of W and B in their dimensions
template <int G, int ST>
sweep_fn su3_lookup(int upd, int ctd, int wi, int bi, int nt);
// gauge group SU(2) (storages ST_SU2_*; W = 1, nt = 0)
sweep_fn sweep_kernel_su2(int gauge, int upd, int st, int ct_double, int W, int B, int nt);

// active != nullptr: the tiles of units whose flag is 0 are skipped and keep
// their partial sums from the last measurement
hipError_t measure(int gauge, int st, unsigned ntiles, hipStream_t s, const gfs::MeasureArgs &a,
                   const int32_t *active = nullptr);
// unit sums -> F = sum / (nc ndir V_u), theta = sum / (nc V_u) (nc: 3 or 2)
hipError_t finalize(int nunits, const gfs::UnitDev *units, const double *partial, int ndir, int nc, double *out,
                    hipStream_t s);
hipError_t finalize_decide(int nunits, const gfs::UnitDev *units, const double *partial, int ndir, int nc,
                           double *out, int32_t *active, int32_t *fp64, double tol, double tail, int32_t *status,
                           uint32_t *counter, hipStream_t s);
hipError_t count_sweep(int ninst, const gfs::InstDev *inst, const int32_t *active, int32_t *sweeps_done,
                       uint64_t *sweep_ix, int32_t n, hipStream_t s);
hipError_t fill_i32(int32_t *p, int32_t v, int n, hipStream_t s);
// reprojection of half-sites [h_lo, h_lo + nh) of nplanes link planes; with
// `active`, half-sites of stopped units (unit0 + h / (Vh / nunits)) are left
// as they are
hipError_t reunit(int st, char *ws, int64_t off, int32_t nplanes, int32_t Vh, int32_t Vp, int32_t h_lo, int32_t nh,
                  const int32_t *active, int32_t unit0, int32_t nunits, hipStream_t s);
hipError_t set_identity(int st, char *ws, int64_t off, int32_t Vh, int32_t Vp, hipStream_t s);
hipError_t convert_in(int st, char *ws, const gfs::InstDev &I, const double *src, int64_t s0, int64_t ns,
                      hipStream_t s);
hipError_t convert_out(int st, const char *ws, const gfs::InstDev &I, double *dst, int64_t s0, int64_t ns, int reunit,
                       hipStream_t s);
hipError_t coulomb_fix(int st, char *ws, const gfs::InstDev &I, hipStream_t s);

// the same for the SU(2) storages (the functions above dispatch to these)
hipError_t measure_su2(int gauge, int st, unsigned ntiles, hipStream_t s, const gfs::MeasureArgs &a,
                       const int32_t *active);
hipError_t reunit_su2(int st, char *ws, int64_t off, int32_t nplanes, int32_t Vp, int32_t h_lo, int32_t nh,
                      const int32_t *active, int32_t unit0, int32_t hper, hipStream_t s);
hipError_t set_identity_su2(int st, char *ws, int64_t off, int32_t Vh, int32_t Vp, hipStream_t s);
hipError_t convert_in_su2(int st, char *ws, const gfs::InstDev &I, const double *src, int64_t s0, int64_t ns,
                          hipStream_t s);
hipError_t convert_out_su2(int st, const char *ws, const gfs::InstDev &I, double *dst, int64_t s0, int64_t ns,
                           int reunit, hipStream_t s);
hipError_t coulomb_fix_su2(int st, char *ws, const gfs::InstDev &I, hipStream_t s);

// no-allocation measurement: the address of this device's fixed scratch
// array (looked up on first use with device `dev` current) and its size; F
// and theta of a natural-order FP64 SU(3) field into out[0], out[1]
hipError_t noalloc_scratch(int dev, double **ptr, size_t *bytes);
hipError_t measure_nat(int gauge, const double *links, const int32_t n[4], double *out, double *scratch,
                       hipStream_t s);

}  // namespace gfl
