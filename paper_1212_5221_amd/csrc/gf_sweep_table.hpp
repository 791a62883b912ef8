// gf_sweep_table.hpp -- the lookup table of the SU(3) half-sweep variants of
// one gauge and one storage, generated from su3_built(): entry sub_index(upd,
// ctd, W, B, nt) is the kernel k_sweep<...> of that variant, or nullptr.
#pragma once

#include <array>
#include <type_traits>
#include <utility>

#include "gf_launch.hpp"
#include "gf_sweep.hpp"
#include "gf_variants.hpp"

namespace gfl {

template <int G, int ST, int I>
sweep_fn su3_entry() {
    constexpr int upd = I % NUPD;
    constexpr int ctd = (I / NUPD) % NCTD;
    constexpr int wi = (I / (NUPD * NCTD)) % NWAVE;
    constexpr int bi = (I / (NUPD * NCTD * NWAVE)) % NBLOCK;
    constexpr int nt = I / (NUPD * NCTD * NWAVE * NBLOCK);
    static_assert(sub_index(upd, ctd, wi, bi, nt) == I, "table index");
    if constexpr (su3_built(G, upd, ST, ctd, wave_of(wi), block_of(bi), nt)) {
        typedef typename std::conditional<ctd == 1, double, float>::type CT;
        return &gfd::k_sweep<G, upd, ST, CT, wave_of(wi), block_of(bi), nt>;
    } else {
        return nullptr;
    }
}

template <int G, int ST, int... I>
std::array<sweep_fn, sizeof...(I)> su3_table(std::integer_sequence<int, I...>) {
    return {{su3_entry<G, ST, I>()...}};
}

template <int G, int ST>
sweep_fn su3_lookup(int upd, int ctd, int wi, int bi, int nt) {
    static const std::array<sweep_fn, NSUB> t = su3_table<G, ST>(std::make_integer_sequence<int, NSUB>{});
    return t[sub_index(upd, ctd, wi, bi, nt)];
}

}  // namespace gfl
