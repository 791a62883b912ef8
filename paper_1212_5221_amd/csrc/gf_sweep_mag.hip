// gf_sweep_mag.hip -- half-sweep kernel variants for the mag gauge.
#include "gf_launch.hpp"
#include "gf_sweep.hpp"

namespace gfl {

sweep_fn sweep_kernel_mag(int upd, int st, int ctd, int W) {
    if (W == 1 && upd == gfs::UPD_OR && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F64R18, double, 1>;
    if (W == 1 && upd == gfs::UPD_OR && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F64R12, double, 1>;
    if (W == 1 && upd == gfs::UPD_OR && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F32R12, double, 1>;
    if (W == 1 && upd == gfs::UPD_OR && st == gfs::ST_F32R12 && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F32R12, float, 1>;
    if (W == 1 && upd == gfs::UPD_MICRO && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F64R18, double, 1>;
    if (W == 1 && upd == gfs::UPD_MICRO && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F64R12, double, 1>;
    if (W == 1 && upd == gfs::UPD_MICRO && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F32R12, double, 1>;
    if (W == 1 && upd == gfs::UPD_MICRO && st == gfs::ST_F32R12 && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F32R12, float, 1>;
    if (W == 1 && upd == gfs::UPD_HEATBATH && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_HEATBATH, gfs::ST_F64R18, double, 1>;
    if (W == 1 && upd == gfs::UPD_HEATBATH && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_HEATBATH, gfs::ST_F64R12, double, 1>;
    if (W == 1 && upd == gfs::UPD_HEATBATH && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_HEATBATH, gfs::ST_F32R12, double, 1>;
    if (W == 1 && upd == gfs::UPD_SR && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_SR, gfs::ST_F64R18, double, 1>;
    if (W == 1 && upd == gfs::UPD_SR && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_SR, gfs::ST_F64R12, double, 1>;
    if (W == 1 && upd == gfs::UPD_SR && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_SR, gfs::ST_F32R12, double, 1>;
    if (W == 2 && upd == gfs::UPD_OR && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F64R18, double, 2>;
    if (W == 2 && upd == gfs::UPD_OR && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F64R12, double, 2>;
    if (W == 2 && upd == gfs::UPD_OR && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F32R12, double, 2>;
    if (W == 2 && upd == gfs::UPD_OR && st == gfs::ST_F32R12 && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F32R12, float, 2>;
    if (W == 2 && upd == gfs::UPD_MICRO && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F64R18, double, 2>;
    if (W == 2 && upd == gfs::UPD_MICRO && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F64R12, double, 2>;
    if (W == 2 && upd == gfs::UPD_MICRO && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F32R12, double, 2>;
    if (W == 2 && upd == gfs::UPD_MICRO && st == gfs::ST_F32R12 && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F32R12, float, 2>;
    if (W == 2 && upd == gfs::UPD_HEATBATH && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_HEATBATH, gfs::ST_F64R18, double, 2>;
    if (W == 2 && upd == gfs::UPD_HEATBATH && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_HEATBATH, gfs::ST_F64R12, double, 2>;
    if (W == 2 && upd == gfs::UPD_HEATBATH && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_HEATBATH, gfs::ST_F32R12, double, 2>;
    if (W == 2 && upd == gfs::UPD_SR && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_SR, gfs::ST_F64R18, double, 2>;
    if (W == 2 && upd == gfs::UPD_SR && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_SR, gfs::ST_F64R12, double, 2>;
    if (W == 2 && upd == gfs::UPD_SR && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_SR, gfs::ST_F32R12, double, 2>;
    if (W == 4 && upd == gfs::UPD_OR && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F64R18, double, 4>;
    if (W == 4 && upd == gfs::UPD_OR && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F64R12, double, 4>;
    if (W == 4 && upd == gfs::UPD_OR && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F32R12, double, 4>;
    if (W == 4 && upd == gfs::UPD_OR && st == gfs::ST_F32R12 && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F32R12, float, 4>;
    if (W == 4 && upd == gfs::UPD_MICRO && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F64R18, double, 4>;
    if (W == 4 && upd == gfs::UPD_MICRO && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F64R12, double, 4>;
    if (W == 4 && upd == gfs::UPD_MICRO && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F32R12, double, 4>;
    if (W == 4 && upd == gfs::UPD_MICRO && st == gfs::ST_F32R12 && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F32R12, float, 4>;
    if (W == 4 && upd == gfs::UPD_HEATBATH && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_HEATBATH, gfs::ST_F64R18, double, 4>;
    if (W == 4 && upd == gfs::UPD_HEATBATH && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_HEATBATH, gfs::ST_F64R12, double, 4>;
    if (W == 4 && upd == gfs::UPD_HEATBATH && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_HEATBATH, gfs::ST_F32R12, double, 4>;
    if (W == 4 && upd == gfs::UPD_SR && st == gfs::ST_F64R18 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_SR, gfs::ST_F64R18, double, 4>;
    if (W == 4 && upd == gfs::UPD_SR && st == gfs::ST_F64R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_SR, gfs::ST_F64R12, double, 4>;
    if (W == 4 && upd == gfs::UPD_SR && st == gfs::ST_F32R12 && ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_SR, gfs::ST_F32R12, double, 4>;
    if (W == 1 && upd == gfs::UPD_OR && st == gfs::ST_F32R12_SP && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F32R12_SP, float, 1>;
    if (W == 1 && upd == gfs::UPD_MICRO && st == gfs::ST_F32R12_SP && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F32R12_SP, float, 1>;
    if (W == 2 && upd == gfs::UPD_OR && st == gfs::ST_F32R12_SP && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F32R12_SP, float, 2>;
    if (W == 2 && upd == gfs::UPD_MICRO && st == gfs::ST_F32R12_SP && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F32R12_SP, float, 2>;
    if (W == 4 && upd == gfs::UPD_OR && st == gfs::ST_F32R12_SP && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_OR, gfs::ST_F32R12_SP, float, 4>;
    if (W == 4 && upd == gfs::UPD_MICRO && st == gfs::ST_F32R12_SP && !ctd) return &gfd::k_sweep<gfs::MAG, gfs::UPD_MICRO, gfs::ST_F32R12_SP, float, 4>;
    return nullptr;
}

}  // namespace gfl
