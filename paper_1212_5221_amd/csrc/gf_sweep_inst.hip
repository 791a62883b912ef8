// gf_sweep_inst.hip -- the SU(3) half-sweep variants of one gauge and one
// link storage.  The build compiles this file once per (GF_GAUGE,
// GF_STORAGE) pair, so the variants compile in parallel.
#include "gf_sweep_table.hpp"

#if !defined(GF_GAUGE) || !defined(GF_STORAGE)
#error "compile with -DGF_GAUGE=<gauge> -DGF_STORAGE=<storage>"
#endif

template gfl::sweep_fn gfl::su3_lookup<GF_GAUGE, GF_STORAGE>(int, int, int, int, int);
