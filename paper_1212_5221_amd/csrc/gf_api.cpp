// gf_api.cpp -- the C ABI of libgf (include/gf.h): handle state, workspace
// carving, instance and unit tables, the Alg. 1 driver with per-unit
// stopping, annealing schedules, HIP-graph capture of the sweep loop,
// kernel timing and the autotuner.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/gf.h"
#include "gf_launch.hpp"
#include "gf_shared.hpp"
#include "gf_variants.hpp"

namespace {

struct InstHost {
    int32_t n[4];
    int64_t V, Vh, Vp;  // sites, half, half rounded up to 16
    int32_t unit0, nunits;
    int64_t links_off, g_off;
};

// Launch shape of one kernel table: W wavefronts per group of 64 sites, B
// threads per block, non-temporal link traffic, XCD-contiguous tile order.
struct Shape {
    int W = 1, B = 256, nt = 0, xcd = 1;
    bool operator==(const Shape &o) const { return W == o.W && B == o.B && nt == o.nt && xcd == o.xcd; }
    int key() const { return ((gfl::wave_index(W) * 4 + gfl::block_index(B)) * 2 + nt) * 2 + xcd; }
};

// Graphs of chunks of sweeps, one per launch pattern: update, chunk length,
// waves per site group, FP64-update variants in use, and the position of
// the chunk relative to the reprojection interval (which sweeps of the chunk
// reproject).  Every setter that changes a kernel argument clears it.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int key_upd = -1, key_n = -1, key_W = -1, key_tail = -1, key_r = -1;
    std::vector<uint8_t> key_live;  // the groups the chunk sweeps (empty: all)
};

// the captured chunks, least recently used first; when full, the least
// recently used one is dropped (a batch whose units stop one by one needs a
// new graph per set of live groups, while the few reprojection positions
// of the current set keep being replayed)
struct GraphCache {
    static constexpr size_t kMax = 32;
    std::vector<GraphEntry> e;
    static void destroy(GraphEntry &g) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    void clear() {
        for (auto &g : e) destroy(g);
        e.clear();
    }
    void drop_oldest() {
        destroy(e.front());
        e.erase(e.begin());
    }
};

}  // namespace

struct gf_ctx {
    int dev = 0;
    hipStream_t stream = nullptr;  // the caller's stream: all work is ordered on it
    hipStream_t cur = nullptr;     // where launches go: `stream`, or `cap` while capturing a graph
    hipStream_t cap = nullptr;     // private stream used only to capture graphs
    std::string err;

    std::vector<InstHost> inst;
    int gauge = GF_LANDAU;
    int nc = 3;  // gauge group SU(nc)
    int storage = GF_F64_R18;
    int reunit_every = 0;
    double tail_theta = 0.0;
    double omega = 1.0, p_sr = 0.5, T = 1.0;
    double sa_T0 = 1.0, sa_T1 = 0.01;
    int sa_steps = 0, sa_micro = 3;
    uint64_t seed = 0;

    bool bound = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;

    // workspace layout (byte offsets)
    size_t off_inst = 0, off_unit = 0, off_tiles[3] = {0, 0, 0}, off_mtiles = 0, off_partial = 0, off_res = 0;
    size_t off_active = 0, off_fp64 = 0, off_sweeps = 0, off_sweepix = 0, off_status = 0, off_stage = 0;
    size_t stage_bytes = 0, need_bytes = 0;
    int nunits = 0, nmtiles = 0;
    int64_t max_tiles = 0;
    std::vector<gfs::UnitDev> units;

    // launch shape per kernel table (0 FP32 update, 1 FP64 update, 2
    // heatbath) and the matching sweep tile tables
    Shape shape[3];
    // persisted autotuning choices: file and its entries (key -> shape)
    std::string tune_path;
    std::map<std::string, Shape> tune_cache;
    int ntiles[3] = {0, 0, 0};
    int force_ctd = -1;  // autotuning: time one precision only

    // host readback (pinned)
    int32_t *hstat = nullptr;
    double *hres = nullptr;
    int32_t *hact = nullptr;  // per-unit active flags of the two check slots (with cache groups)

    // timing: inside gf_sweep every time_every-th chunk runs plain launches,
    // each bracketed by events (time_now), the others replay graphs;
    // elsewhere every launch is timed
    bool timing = false;
    int time_every = 1;
    uint64_t chunk_seq = 0;
    bool time_now = true;
    std::vector<hipEvent_t> ev_pool;
    struct Pending {
        hipEvent_t e0, e1;
        int ctd;  // compute precision of the timed launch: 0 FP32, 1 FP64
    };
    std::vector<Pending> ev_pending;
    double t_sum_ms[2] = {0.0, 0.0};
    int64_t t_count[2] = {0, 0};

    bool use_graph = true;
    GraphCache graph;
    // Infinity-Cache groups: consecutive units whose working sets together
    // fit cache_budget bytes; inside gf_sweep each group runs the whole chunk
    // of sweeps before the next group starts (units are independent, so
    // every unit's sequence of sweeps is unchanged)
    int64_t cache_budget = (int64_t)224 << 20;
    std::vector<int> grp_u0;         // group g = units [grp_u0[g], grp_u0[g + 1])
    // inside gf_sweep, per group, from the last check read: 0 every unit
    // stopped, 1 some stopped, 2 all active (empty: outside gf_sweep, sweep
    // every group as all active).  Units only stop at checks, so a group
    // whose units have all stopped is skipped (its kernels would exit at
    // once, but their launches still cost time), and a group with stopped
    // units is launched in the linear tile order (see launch_half).
    std::vector<uint8_t> grp_live;
    std::vector<int32_t> tile_u0[3]; // per tile table: first tile of each unit (+ end)

    // from the last check: active units, of which in the FP64 tail
    int n_active = 0, n_tail = 0;
    hipEvent_t chk_ev[2] = {nullptr, nullptr};
};

namespace {

// message of the last failure without a handle (gf_create, gf_measure_noalloc), per host thread
thread_local std::string g_create_error;

int fail(gf_ctx *h, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_create_error = buf;
    return code;
}

#define HIPCHK(h, call)                                                                                   \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return fail((h), GF_E_HIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                            \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// 16-byte chunks per stored link
int nchunks(const gf_ctx *h) {
    if (h->nc == 2) return (h->storage == GF_MIXED_F32_R12 || h->storage == GF_F32_R12) ? 1 : 2;
    switch (h->storage) {
    case GF_F64_R18:
        return 9;
    case GF_F64_R12:
        return 6;
    default:
        return 3;
    }
}

// kernel storage code; SU(2) keeps 4 reals per link in FP64, or in FP32
// for the mixed and single-precision policies
int st_code(const gf_ctx *h) {
    if (h->nc == 2)
        return (h->storage == GF_MIXED_F32_R12 || h->storage == GF_F32_R12) ? gfs::ST_SU2_F32 : gfs::ST_SU2_F64;
    switch (h->storage) {
    case GF_F64_R18:
        return gfs::ST_F64R18;
    case GF_F64_R12:
        return gfs::ST_F64R12;
    default:
        return gfs::ST_F32R12;
    }
}

int ndir(const gf_ctx *h) { return h->gauge == GF_COULOMB ? 3 : 4; }

// reals per site in the natural layout: 4 links of nc x nc complex entries
int64_t site_reals(const gf_ctx *h) { return 8 * (int64_t)h->nc * h->nc; }

int upd_code(int update) {
    switch (update) {
    case GF_OR:
        return gfs::UPD_OR;
    case GF_MICRO:
        return gfs::UPD_MICRO;
    case GF_SR:
        return gfs::UPD_SR;
    case GF_HEATBATH:
        return gfs::UPD_HEATBATH;
    default:
        return -1;
    }
}

template <typename T>
T *wsp(gf_ctx *h, size_t off) {
    return reinterpret_cast<T *>(h->ws + off);
}

// compute the layout; with ws == nullptr only the size
void plan_layout(gf_ctx *h) {
    size_t off = 0;
    const int nch = nchunks(h);
    int unit = 0;
    for (auto &I : h->inst) {
        I.links_off = (int64_t)off;
        off += align256((size_t)8 * nch * I.Vp * 16);
        I.unit0 = unit;
        I.nunits = (h->gauge == GF_COULOMB) ? I.n[0] : 1;
        unit += I.nunits;
        if (h->gauge == GF_COULOMB) {
            I.g_off = (int64_t)off;
            off += align256((size_t)2 * nch * I.Vp * 16);
        } else {
            I.g_off = -1;
        }
    }
    h->nunits = unit;
    h->units.clear();
    int mt = 0;
    int64_t tiles_min = 0;
    for (size_t i = 0; i < h->inst.size(); ++i) {
        const InstHost &I = h->inst[i];
        for (int k = 0; k < I.nunits; ++k) {
            gfs::UnitDev u;
            u.inst = (int32_t)i;
            if (h->gauge == GF_COULOMB) {
                const int32_t hs = (int32_t)(I.Vh / I.n[0]);
                u.t = k;
                u.h0 = k * hs;
                u.n = hs;
            } else {
                u.t = -1;
                u.h0 = 0;
                u.n = (int32_t)I.Vh;
            }
            const int per = (u.n + gfs::MTILE_SITES - 1) / gfs::MTILE_SITES;
            u.mtile0 = mt;
            mt += per;
            u.mtile1 = mt;
            tiles_min += (u.n + 63) / 64;
            h->units.push_back(u);
        }
    }
    h->nmtiles = mt;
    h->max_tiles = tiles_min;
    h->off_inst = off;
    off += align256(sizeof(gfs::InstDev) * h->inst.size());
    h->off_unit = off;
    off += align256(sizeof(gfs::UnitDev) * h->nunits);
    for (int v = 0; v < 3; ++v) {
        h->off_tiles[v] = off;
        off += align256(sizeof(gfs::Tile) * (size_t)h->max_tiles);
    }
    h->off_mtiles = off;
    off += align256(sizeof(gfs::MTile) * (size_t)h->nmtiles);
    h->off_partial = off;
    off += align256(sizeof(double) * 4 * (size_t)h->nmtiles);
    h->off_res = off;
    off += align256(sizeof(double) * 4 * (size_t)h->nunits);
    h->off_active = off;
    off += align256(sizeof(int32_t) * h->nunits);
    h->off_fp64 = off;
    off += align256(sizeof(int32_t) * h->nunits);
    h->off_sweeps = off;
    off += align256(sizeof(int32_t) * h->nunits);
    h->off_sweepix = off;
    off += align256(sizeof(uint64_t) * h->inst.size());
    h->off_status = off;
    off += 256;
    // staging for host uploads/downloads: up to 32 MiB, at least one site
    int64_t maxV = 0;
    for (auto &I : h->inst) maxV = std::max(maxV, I.V);
    h->stage_bytes = align256(std::min<size_t>((size_t)32 << 20, (size_t)maxV * 8 * site_reals(h)));
    h->off_stage = off;
    off += h->stage_bytes;
    h->need_bytes = off;
}

gfs::InstDev inst_dev(const InstHost &I) {
    gfs::InstDev d;
    for (int k = 0; k < 4; ++k) d.n[k] = I.n[k];
    d.Vh = (int32_t)I.Vh;
    d.unit0 = I.unit0;
    d.nunits = I.nunits;
    d.Vp = (int32_t)I.Vp;
    d.links_off = I.links_off;
    d.g_off = I.g_off;
    return d;
}

// compute precision of the heatbath kernels: FP32 on FP32 storage (SU(3);
// the local algebra in FP32 as for overrelaxation, the sample drawn in FP64,
// G applied in FP64), unless the FP64 update is requested throughout
int heatbath_ctd(const gf_ctx *h) {
    const bool f32 = h->storage == GF_MIXED_F32_R12 || h->storage == GF_F32_R12;
    return (h->nc == 3 && f32 && h->tail_theta < 1e300) ? 0 : 1;
}

// sweep tile table `tab` (0 FP32 update, 1 FP64 update, 2 heatbath) for the
// launch shape `sh`: tiles of B / W sites
int build_tiles(gf_ctx *h, int tab, const Shape &sh) {
    const int spb = sh.B / sh.W;
    std::vector<gfs::Tile> t;
    h->tile_u0[tab].assign(h->nunits + 1, 0);
    for (int u = 0; u < h->nunits; ++u) {
        h->tile_u0[tab][u] = (int32_t)t.size();
        for (int32_t j = 0; j < h->units[u].n; j += spb) t.push_back({u, j});
    }
    h->tile_u0[tab][h->nunits] = (int32_t)t.size();
    if ((int64_t)t.size() > h->max_tiles) return fail(h, GF_E_INVALID, "tile table overflow");
    HIPCHK(h, hipMemcpyAsync(h->ws + h->off_tiles[tab], t.data(), sizeof(gfs::Tile) * t.size(), hipMemcpyHostToDevice,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->ntiles[tab] = (int)t.size();
    h->shape[tab] = sh;
    h->graph.clear();
    return GF_OK;
}

// the kernel that table `tab` launches for the OR update (heatbath table:
// the heatbath) with shape sh, nullptr if not built.  A shape of the FP64
// table must also have the stochastic-relaxation variant (cached), which
// runs with that table's shape.
gfl::sweep_fn table_kernel(const gf_ctx *h, int tab, const Shape &sh) {
    const int st = st_code(h);
    const int upd = (tab == 2) ? gfs::UPD_HEATBATH : gfs::UPD_OR;
    const int ctd = (tab == 2) ? heatbath_ctd(h) : (tab == 0) ? 0 : 1;
    const int kst = (h->storage == GF_F32_R12 && tab == 0)
                        ? (h->nc == 2 ? (int)gfs::ST_SU2_F32_SP : (int)gfs::ST_F32R12_SP)
                        : st;
    if (tab == 1 && !gfl::sweep_kernel(h->gauge, gfs::UPD_SR, st, 1, sh.W, sh.B, 0)) return nullptr;
    return gfl::sweep_kernel(h->gauge, upd, kst, ctd, sh.W, sh.B, sh.nt);
}

// every shape table `tab` can launch
std::vector<Shape> table_shapes(const gf_ctx *h, int tab) {
    std::vector<Shape> v;
    for (int xcd = 1; xcd >= 0; --xcd)
        for (int nt = 0; nt < gfl::NNT; ++nt)
            for (int wi = 0; wi < gfl::NWAVE; ++wi)
                for (int bi = 0; bi < gfl::NBLOCK; ++bi) {
                    Shape sh;
                    sh.W = gfl::wave_of(wi);
                    sh.B = gfl::block_of(bi);
                    sh.nt = nt;
                    sh.xcd = xcd;
                    if (table_kernel(h, tab, sh)) v.push_back(sh);
                }
    return v;
}

// default shape: 256 threads, cached, XCD order; W for the FP32 update 1,
// for the FP64 update the largest available of 4, 2, 1 (fewer links per
// wavefront, more waves in flight); heatbath (measured at 32^4): 1 on FP32
// storage, 2 on FP64-12, 4 on FP64-18 where available
Shape default_shape(const gf_ctx *h, int tab) {
    const int st = st_code(h);
    Shape sh;
    if (tab == 0) return sh;
    const int first = (tab == 2) ? ((st == gfs::ST_F32R12) ? 1 : (st == gfs::ST_F64R12 ? 2 : 4)) : 4;
    for (int W = first; W >= 1; W /= 2) {
        sh.W = W;
        if (table_kernel(h, tab, sh)) return sh;
    }
    sh.W = 1;
    return sh;
}

int check_bound(gf_ctx *h) {
    if (!h) return GF_E_INVALID;
    if (!h->bound) return fail(h, GF_E_STATE, "no workspace bound (call gf_bind_workspace first)");
    return GF_OK;
}

int check_unbound(gf_ctx *h) {
    if (!h) return GF_E_INVALID;
    if (h->bound) return fail(h, GF_E_STATE, "configuration is fixed once a workspace is bound");
    return GF_OK;
}

// bytes a unit's sweeps touch: 8 link planes over its half-sites (Coulomb:
// 6 spatial planes and the 2 accumulator planes)
int64_t unit_bytes(const gf_ctx *h, int u) {
    return 8 * (int64_t)h->units[u].n * nchunks(h) * 16;
}

void build_groups(gf_ctx *h) {
    h->grp_u0.assign(1, 0);
    int64_t acc = 0;
    for (int u = 0; u < h->nunits; ++u) {
        const int64_t b = unit_bytes(h, u);
        if (h->cache_budget > 0 && u > h->grp_u0.back() && acc + b > h->cache_budget) {
            h->grp_u0.push_back(u);
            acc = 0;
        }
        acc += b;
    }
    if (h->cache_budget <= 0) h->grp_u0.assign(1, 0);
    h->grp_u0.push_back(h->nunits);
}

int ngroups(const gf_ctx *h) { return (int)h->grp_u0.size() - 1; }

// grp < 0: every tile; else the tiles of group grp
gfs::SweepArgs sweep_args(gf_ctx *h, int parity, int fp64_select, double T, int tab, int sweep_off, int grp,
                          int *ntiles) {
    gfs::SweepArgs a;
    a.ws = h->ws;
    a.inst = wsp<gfs::InstDev>(h, h->off_inst);
    a.unit = wsp<gfs::UnitDev>(h, h->off_unit);
    a.tiles = wsp<gfs::Tile>(h, h->off_tiles[tab]);
    *ntiles = h->ntiles[tab];
    if (grp >= 0) {
        const int32_t t0 = h->tile_u0[tab][h->grp_u0[grp]], t1 = h->tile_u0[tab][h->grp_u0[grp + 1]];
        a.tiles += t0;
        *ntiles = t1 - t0;
    }
    a.active = wsp<int32_t>(h, h->off_active);
    a.fp64 = wsp<int32_t>(h, h->off_fp64);
    a.sweep_ix = wsp<uint64_t>(h, h->off_sweepix);
    a.parity = parity;
    a.fp64_select = fp64_select;
    a.sweep_off = sweep_off;
    a.xcd_order = 1;
    a.omega = h->omega;
    a.T = T;
    a.p_sr = h->p_sr;
    a.seed = h->seed;
    return a;
}

hipEvent_t take_event(gf_ctx *h) {
    if (!h->ev_pool.empty()) {
        hipEvent_t e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int drain_timing(gf_ctx *h) {
    if (h->ev_pending.empty()) return GF_OK;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (auto &p : h->ev_pending) {
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, p.e0, p.e1));
        h->t_sum_ms[p.ctd] += ms;
        h->t_count[p.ctd] += 1;
        h->ev_pool.push_back(p.e0);
        h->ev_pool.push_back(p.e1);
    }
    h->ev_pending.clear();
    return GF_OK;
}

// one half-sweep of update `upd` (gfs code) at temperature T on all active units
int launch_half(gf_ctx *h, int upd, int parity, double T, bool capturing, int sweep_off, int grp = -1) {
    const int st = st_code(h);
    const bool mixed = (h->storage == GF_MIXED_F32_R12);
    const bool single = (h->storage == GF_F32_R12);
    const bool hb = (upd == gfs::UPD_HEATBATH || upd == gfs::UPD_SR);
    // compute precision: FP64 storage -> double; mixed -> float (+ double tail)
    // ctd: compute precision of the update (0 FP32, 1 FP64); tab: tile table
    struct L {
        int ctd, sel, tab;
    } launches[2];
    int nl = 0;
    if (h->force_ctd >= 0) {
        launches[nl++] = {h->force_ctd, -1, h->force_ctd};
    } else if (upd == gfs::UPD_HEATBATH) {
        launches[nl++] = {heatbath_ctd(h), -1, 2};
    } else if (single && !hb) {
        launches[nl++] = {0, -1, 0};
    } else if (!mixed || hb) {
        launches[nl++] = {1, -1, 1};
    } else if (h->tail_theta > 0.0) {
        // only the variants some active unit needs (counts of the last check)
        if (h->n_tail == 0)
            launches[nl++] = {0, -1, 0};
        else if (h->n_tail >= h->n_active)
            launches[nl++] = {1, -1, 1};
        else {
            launches[nl++] = {0, 0, 0};
            launches[nl++] = {1, 1, 1};
        }
    } else {
        launches[nl++] = {0, -1, 0};
    }
    for (int k = 0; k < nl; ++k) {
        const int ctd = launches[k].ctd, tab = launches[k].tab;
        // single precision: the FP32-update kernels that also apply G in FP32
        // (the heatbath applies G in FP64 on both FP32 storages)
        const int kst = (single && ctd == 0 && upd != gfs::UPD_HEATBATH)
                            ? (h->nc == 2 ? (int)gfs::ST_SU2_F32_SP : (int)gfs::ST_F32R12_SP)
                            : st;
        const Shape &sh = h->shape[tab];
        // the random updates have cached variants only
        gfl::sweep_fn fn = gfl::sweep_kernel(h->gauge, upd, kst, ctd, sh.W, sh.B, gfl::is_random(upd) ? 0 : sh.nt);
        if (!fn)
            return fail(h, GF_E_INVALID, "no kernel variant for gauge %d update %d storage %d W %d B %d", h->gauge,
                        upd, h->storage, sh.W, sh.B);
        int nt = 0;
        gfs::SweepArgs a = sweep_args(h, parity, launches[k].sel, T, tab, sweep_off, grp, &nt);
        // The XCD-contiguous order hands each XCD a contiguous eighth of the
        // tiles.  When only some units of the launch do work (stopped units,
        // or the units of the other precision, whose blocks exit at once),
        // the working tiles would crowd onto a few XCDs; the linear order
        // deals consecutive blocks round the XCDs and spreads them.
        const bool uniform =
            launches[k].sel < 0 && (h->grp_live.empty() || h->grp_live[grp < 0 ? 0 : grp] == 2);
        a.xcd_order = sh.xcd && uniform;
        if (nt <= 0) continue;
        const bool tm = h->timing && !capturing && h->time_now;
        if (tm) {
            // the launch itself records its start and stop events
            hipEvent_t e0 = take_event(h), e1 = take_event(h);
            if (!e0 || !e1) return fail(h, GF_E_HIP, "hipEventCreate failed");
            void *args[] = {&a};
            HIPCHK(h, hipExtLaunchKernel(reinterpret_cast<const void *>(fn), dim3((unsigned)nt), dim3((unsigned)sh.B),
                                         args, 0, h->cur, e0, e1, 0));
            h->ev_pending.push_back({e0, e1, launches[k].ctd});
            if (h->ev_pending.size() > 4096) {
                int rc = drain_timing(h);
                if (rc) return rc;
            }
        } else {
            fn<<<dim3((unsigned)nt), dim3((unsigned)sh.B), 0, h->cur>>>(a);
            HIPCHK(h, hipGetLastError());
        }
    }
    return GF_OK;
}

// reprojection of the links (and Coulomb accumulator) of units [u0, u1);
// inside gf_sweep (only_active) stopped units are skipped, so they keep the
// links their stopping check measured
int launch_reunit_units(gf_ctx *h, bool only_active, int u0, int u1) {
    const int st = st_code(h);
    const int32_t *act = only_active ? wsp<int32_t>(h, h->off_active) : nullptr;
    for (auto &I : h->inst) {
        const int a = std::max(u0, (int)I.unit0), b = std::min(u1, (int)(I.unit0 + I.nunits));
        if (a >= b) continue;
        const int32_t h_lo = h->units[a].h0, h_hi = h->units[b - 1].h0 + h->units[b - 1].n;
        HIPCHK(h, gfl::reunit(st, h->ws, I.links_off, 8, (int32_t)I.Vh, (int32_t)I.Vp, h_lo, h_hi - h_lo, act,
                              I.unit0, I.nunits, h->cur));
        if (I.g_off >= 0)
            HIPCHK(h, gfl::reunit(st, h->ws, I.g_off, 2, (int32_t)I.Vh, (int32_t)I.Vp, h_lo, h_hi - h_lo, act,
                                  I.unit0, I.nunits, h->cur));
    }
    return GF_OK;
}

int launch_reunit_all(gf_ctx *h, bool only_active) { return launch_reunit_units(h, only_active, 0, h->nunits); }

// one full sweep (both parities) [+ reprojection]; sweep_off is the sweep's
// position in its chunk (random counter offset), counted by count_chunk
int launch_sweep(gf_ctx *h, int upd, double T, bool reunit_now, bool capturing, int sweep_off, int grp = -1) {
    for (int p = 0; p < 2; ++p) {
        int rc = launch_half(h, upd, p, T, capturing, sweep_off, grp);
        if (rc) return rc;
    }
    if (!reunit_now) return GF_OK;
    if (grp < 0) return launch_reunit_all(h, true);
    return launch_reunit_units(h, true, h->grp_u0[grp], h->grp_u0[grp + 1]);
}

// n sweeps of every unit, chunk positions k0 .. k0 + n - 1; with several
// cache groups, group by group
int enqueue_chunk(gf_ctx *h, int upd, int n, int k0, bool capturing) {
    const int R = h->reunit_every;
    const int ng = ngroups(h);
    for (int g = 0; g < ng; ++g) {
        if (ng > 1 && !h->grp_live.empty() && h->grp_live[g] == 0) continue;  // every unit has stopped
        for (int i = 0; i < n; ++i) {
            const bool rn = (R > 0) && ((k0 + i + 1) % R == 0);
            int rc = launch_sweep(h, upd, h->T, rn, capturing, i, ng > 1 ? g : -1);
            if (rc) return rc;
        }
    }
    return GF_OK;
}

// per group: 0 no active unit, 1 some, 2 all, from per-unit active flags
void set_live_groups(gf_ctx *h, const int32_t *active) {
    const int ng = ngroups(h);
    for (int g = 0; g < ng; ++g) {
        int n = 0;
        for (int u = h->grp_u0[g]; u < h->grp_u0[g + 1]; ++u) n += active[u] != 0;
        h->grp_live[g] = (n == 0) ? 0 : (n == h->grp_u0[g + 1] - h->grp_u0[g] ? 2 : 1);
    }
}

// after a chunk of n sweeps: sweeps_done and the random-stream index
int count_chunk(gf_ctx *h, int n) {
    HIPCHK(h, gfl::count_sweep((int)h->inst.size(), wsp<gfs::InstDev>(h, h->off_inst), wsp<int32_t>(h, h->off_active),
                               wsp<int32_t>(h, h->off_sweeps), wsp<uint64_t>(h, h->off_sweepix), n, h->cur));
    return GF_OK;
}

// F / theta of every unit; with decide, also the stopping decision (one
// finalize kernel whose last block decides).  only_active (inside gf_sweep):
// the tiles of stopped units are not read again, their partial sums from
// the measurement that stopped them stand (their links have not changed)
int launch_measure(gf_ctx *h, int with_unitarity, bool decide = false, double tol = 0.0, bool only_active = false) {
    gfs::MeasureArgs a;
    a.ws = h->ws;
    a.inst = wsp<gfs::InstDev>(h, h->off_inst);
    a.unit = wsp<gfs::UnitDev>(h, h->off_unit);
    a.tiles = wsp<gfs::MTile>(h, h->off_mtiles);
    a.partial = wsp<double>(h, h->off_partial);
    a.with_unitarity = with_unitarity;
    HIPCHK(h, gfl::measure(h->gauge, st_code(h), (unsigned)h->nmtiles, h->cur, a,
                           only_active ? wsp<int32_t>(h, h->off_active) : nullptr));
    if (!decide) {
        HIPCHK(h, gfl::finalize(h->nunits, wsp<gfs::UnitDev>(h, h->off_unit), wsp<double>(h, h->off_partial),
                                ndir(h), h->nc, wsp<double>(h, h->off_res), h->cur));
        return GF_OK;
    }
    const double tail = (h->storage == GF_MIXED_F32_R12) ? h->tail_theta : 0.0;
    HIPCHK(h, gfl::finalize_decide(h->nunits, wsp<gfs::UnitDev>(h, h->off_unit), wsp<double>(h, h->off_partial),
                                   ndir(h), h->nc, wsp<double>(h, h->off_res), wsp<int32_t>(h, h->off_active),
                                   wsp<int32_t>(h, h->off_fp64), tol, tail, wsp<int32_t>(h, h->off_status),
                                   wsp<uint32_t>(h, h->off_status + 16), h->cur));
    return GF_OK;
}


int coulomb_finish(gf_ctx *h) {
    if (h->gauge != GF_COULOMB) return GF_OK;
    const int st = st_code(h);
    for (auto &I : h->inst) {
        const gfs::InstDev d = inst_dev(I);
        HIPCHK(h, gfl::coulomb_fix(st, h->ws, d, h->cur));
        HIPCHK(h, gfl::set_identity(st, h->ws, I.g_off, (int32_t)I.Vh, (int32_t)I.Vp, h->cur));
    }
    return GF_OK;
}

// run `n` sweeps starting at sweep count k0 (of this gf_sweep call)
int run_sweeps(gf_ctx *h, int upd, int n, int k0, bool chunk_is_full) {
    const int R = h->reunit_every;
    // with timing on, every time_every-th chunk is a timing sample of plain
    // launches; graphs replay the others
    bool sample = false;
    if (h->timing) sample = (h->chunk_seq++ % (uint64_t)h->time_every) == 0;
    const bool graph_ok = h->use_graph && !sample && chunk_is_full;
    if (!graph_ok) {
        h->time_now = sample;
        int rc = enqueue_chunk(h, upd, n, k0, false);
        h->time_now = true;
        if (rc) return rc;
        return count_chunk(h, n);
    }
    int tailkey = 0;
    if (h->storage == GF_MIXED_F32_R12 && h->tail_theta > 0.0)
        tailkey = (h->n_tail == 0) ? 1 : (h->n_tail >= h->n_active ? 2 : 3);
    const int wkey = (h->shape[0].key() * 64 + h->shape[1].key()) * 64 + h->shape[2].key();
    // which sweeps of the chunk reproject: none or one (R >= n, keyed by the
    // position), or a pattern fixed by k0 mod R (R < n)
    int rkey = -1;
    if (R > 0) {
        if (R >= n) {
            const int p = R - 1 - k0 % R;
            rkey = (p < n) ? p : -1;
        } else {
            rkey = n + k0 % R;
        }
    }
    GraphCache &gc = h->graph;
    GraphEntry *g = nullptr;
    for (size_t i = 0; i < gc.e.size(); ++i) {
        const GraphEntry &x = gc.e[i];
        if (x.key_upd == upd && x.key_n == n && x.key_W == wkey && x.key_tail == tailkey && x.key_r == rkey &&
            x.key_live == h->grp_live) {
            std::rotate(gc.e.begin() + i, gc.e.begin() + i + 1, gc.e.end());  // now the most recent
            g = &gc.e.back();
            break;
        }
    }
    if (!g) {
        if (gc.e.size() >= GraphCache::kMax) gc.drop_oldest();
        if (!h->cap) HIPCHK(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        HIPCHK(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        h->cur = h->cap;
        int rc = enqueue_chunk(h, upd, n, k0, true);
        if (rc == GF_OK) rc = count_chunk(h, n);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(h->cap, &gr);
        h->cur = h->stream;
        if (rc) {
            if (gr) (void)hipGraphDestroy(gr);
            return rc;
        }
        if (e != hipSuccess) return fail(h, GF_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        GraphEntry ne;
        ne.graph = gr;
        hipError_t ie = hipGraphInstantiate(&ne.exec, gr, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(gr);
            return fail(h, GF_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
        }
        ne.key_upd = upd;
        ne.key_n = n;
        ne.key_W = wkey;
        ne.key_tail = tailkey;
        ne.key_r = rkey;
        ne.key_live = h->grp_live;
        gc.e.push_back(ne);
        g = &gc.e.back();
    }
    HIPCHK(h, hipGraphLaunch(g->exec, h->stream));
    return GF_OK;
}

int fetch_sweeps_done(gf_ctx *h, int32_t *sweeps_done) {
    if (!sweeps_done) return GF_OK;
    HIPCHK(h, hipMemcpyAsync(sweeps_done, h->ws + h->off_sweeps, sizeof(int32_t) * h->nunits, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return GF_OK;
}

int check_inst(gf_ctx *h, int32_t inst) {
    if (inst < 0 || inst >= (int32_t)h->inst.size()) return fail(h, GF_E_INVALID, "no instance %d", inst);
    return GF_OK;
}

}  // namespace

namespace gfl {
template <int G>
static sweep_fn su3_by_storage(int upd, int st, int ctd, int wi, int bi, int nt) {
    if (st == gfs::ST_F64R18) return su3_lookup<G, gfs::ST_F64R18>(upd, ctd, wi, bi, nt);
    if (st == gfs::ST_F64R12) return su3_lookup<G, gfs::ST_F64R12>(upd, ctd, wi, bi, nt);
    if (st == gfs::ST_F32R12) return su3_lookup<G, gfs::ST_F32R12>(upd, ctd, wi, bi, nt);
    return su3_lookup<G, gfs::ST_F32R12_SP>(upd, ctd, wi, bi, nt);
}

sweep_fn sweep_kernel(int gauge, int upd, int st, int ct_double, int W, int B, int nt) {
    if (gfs::is_su2(st)) return sweep_kernel_su2(gauge, upd, st, ct_double, W, B, nt);
    if (upd < 0 || upd >= NUPD || !su3_built(gauge, upd, st, ct_double, W, B, nt)) return nullptr;
    const int wi = wave_index(W), bi = block_index(B);
    if (gauge == gfs::LANDAU) return su3_by_storage<gfs::LANDAU>(upd, st, ct_double, wi, bi, nt);
    if (gauge == gfs::COULOMB) return su3_by_storage<gfs::COULOMB>(upd, st, ct_double, wi, bi, nt);
    return su3_by_storage<gfs::MAG>(upd, st, ct_double, wi, bi, nt);
}
}  // namespace gfl

// ======================================================================== ABI
extern "C" {

int gf_create(gf_handle *out, int hip_device, void *hip_stream) {
    if (!out) return fail(nullptr, GF_E_INVALID, "gf_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return fail(nullptr, GF_E_HIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= ndev) return fail(nullptr, GF_E_INVALID, "no HIP device %d", hip_device);
    e = hipSetDevice(hip_device);
    if (e != hipSuccess) return fail(nullptr, GF_E_HIP, "hipSetDevice: %s", hipGetErrorString(e));
    gf_ctx *h = new gf_ctx();
    h->dev = hip_device;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    h->cur = h->stream;
    e = hipHostMalloc(reinterpret_cast<void **>(&h->hstat), 16 * sizeof(int32_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete h;
        return fail(nullptr, GF_E_HIP, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    *out = h;
    return GF_OK;
}

void gf_destroy(gf_handle h) {
    if (!h) return;
    (void)hipSetDevice(h->dev);
    if (!h->ev_pending.empty()) (void)hipStreamSynchronize(h->stream);
    h->graph.clear();
    for (auto &p : h->ev_pending) {
        (void)hipEventDestroy(p.e0);
        (void)hipEventDestroy(p.e1);
    }
    for (auto e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->hstat) (void)hipHostFree(h->hstat);
    if (h->hres) (void)hipHostFree(h->hres);
    if (h->hact) (void)hipHostFree(h->hact);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    for (auto e : h->chk_ev)
        if (e) (void)hipEventDestroy(e);
    delete h;
}

const char *gf_last_error(gf_handle h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int gf_add_instance(gf_handle h, const int32_t dims[4], int32_t *inst) {
    int rc = check_unbound(h);
    if (rc) return rc;
    if (!dims) return fail(h, GF_E_INVALID, "dims is NULL");
    int64_t V = 1;
    for (int k = 0; k < 4; ++k) {
        if (dims[k] < 2 || (dims[k] & 1))
            return fail(h, GF_E_DIMS, "extent %d of dimension %d is not even and >= 2", dims[k], k);
        V *= dims[k];
    }
    if (V / 2 >= ((int64_t)1 << 28)) return fail(h, GF_E_DIMS, "lattice too large (%lld sites)", (long long)V);
    InstHost I;
    for (int k = 0; k < 4; ++k) I.n[k] = dims[k];
    I.V = V;
    I.Vh = V / 2;
    I.Vp = (I.Vh + 15) / 16 * 16;
    I.unit0 = I.nunits = 0;
    I.links_off = I.g_off = 0;
    h->inst.push_back(I);
    if (inst) *inst = (int32_t)h->inst.size() - 1;
    return GF_OK;
}

int gf_set_gauge(gf_handle h, int gauge) {
    int rc = check_unbound(h);
    if (rc) return rc;
    if (gauge != GF_LANDAU && gauge != GF_COULOMB && gauge != GF_MAG) return fail(h, GF_E_INVALID, "bad gauge %d", gauge);
    h->gauge = gauge;
    return GF_OK;
}

int gf_set_group(gf_handle h, int nc) {
    int rc = check_unbound(h);
    if (rc) return rc;
    if (nc != 2 && nc != 3) return fail(h, GF_E_INVALID, "gauge group SU(%d) is not supported (2 or 3)", nc);
    h->nc = nc;
    return GF_OK;
}

int gf_set_precision(gf_handle h, int storage, int32_t reunit_every, double fp64_tail_theta) {
    int rc = check_unbound(h);
    if (rc) return rc;
    if (storage != GF_F64_R18 && storage != GF_F64_R12 && storage != GF_MIXED_F32_R12 && storage != GF_F32_R12)
        return fail(h, GF_E_INVALID, "bad storage %d", storage);
    if (reunit_every < 0) return fail(h, GF_E_INVALID, "reunit_every < 0");
    if (!(fp64_tail_theta >= 0.0)) return fail(h, GF_E_INVALID, "fp64_tail_theta must be >= 0");
    h->storage = storage;
    h->reunit_every = reunit_every;
    h->tail_theta = fp64_tail_theta;
    return GF_OK;
}

int gf_workspace_size(gf_handle h, size_t *bytes) {
    if (!h || !bytes) return fail(h, GF_E_INVALID, "NULL argument");
    if (h->inst.empty()) return fail(h, GF_E_STATE, "no instance added");
    plan_layout(h);
    *bytes = h->need_bytes;
    return GF_OK;
}

int gf_bind_workspace(gf_handle h, void *dev_ptr, size_t bytes) {
    int rc = check_unbound(h);
    if (rc) return rc;
    if (h->inst.empty()) return fail(h, GF_E_STATE, "no instance added");
    if (!dev_ptr) return fail(h, GF_E_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_ptr) & 255) return fail(h, GF_E_NOMEM, "workspace not 256-byte aligned");
    plan_layout(h);
    if (bytes < h->need_bytes)
        return fail(h, GF_E_NOMEM, "workspace of %zu bytes, %zu needed", bytes, h->need_bytes);
    HIPCHK(h, hipSetDevice(h->dev));
    h->ws = reinterpret_cast<char *>(dev_ptr);
    h->ws_bytes = bytes;
    std::vector<gfs::InstDev> idv;
    for (auto &I : h->inst) idv.push_back(inst_dev(I));
    std::vector<gfs::MTile> mt;
    for (int u = 0; u < h->nunits; ++u) {
        const gfs::UnitDev &U = h->units[u];
        for (int32_t j = 0; j < U.n; j += gfs::MTILE_SITES) mt.push_back({u, 0, j, 0});
    }
    HIPCHK(h, hipMemcpyAsync(h->ws + h->off_inst, idv.data(), sizeof(gfs::InstDev) * idv.size(), hipMemcpyHostToDevice,
                             h->stream));
    HIPCHK(h, hipMemcpyAsync(h->ws + h->off_unit, h->units.data(), sizeof(gfs::UnitDev) * h->units.size(),
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->ws + h->off_mtiles, mt.data(), sizeof(gfs::MTile) * mt.size(), hipMemcpyHostToDevice,
                             h->stream));
    std::vector<uint64_t> zero(h->inst.size(), 0);
    HIPCHK(h, hipMemcpyAsync(h->ws + h->off_sweepix, zero.data(), sizeof(uint64_t) * zero.size(), hipMemcpyHostToDevice,
                             h->stream));
    HIPCHK(h, gfl::fill_i32(wsp<int32_t>(h, h->off_active), 1, h->nunits, h->stream));
    // FP64 tail flags: before any measurement theta is unknown; a threshold of
    // 1e300 or more means "always FP64"
    HIPCHK(h, gfl::fill_i32(wsp<int32_t>(h, h->off_fp64), h->tail_theta >= 1e300 ? 1 : 0, h->nunits, h->stream));
    HIPCHK(h, gfl::fill_i32(wsp<int32_t>(h, h->off_sweeps), 0, h->nunits, h->stream));
    HIPCHK(h, gfl::fill_i32(wsp<int32_t>(h, h->off_status), 0, 8, h->stream));  // status + finalize counter
    const int st = st_code(h);
    for (auto &I : h->inst)
        if (I.g_off >= 0) HIPCHK(h, gfl::set_identity(st, h->ws, I.g_off, (int32_t)I.Vh, (int32_t)I.Vp, h->stream));
    if (h->hres) (void)hipHostFree(h->hres);
    HIPCHK(h, hipHostMalloc(reinterpret_cast<void **>(&h->hres), sizeof(double) * 4 * h->nunits, hipHostMallocDefault));
    h->n_active = h->nunits;
    h->n_tail = (h->tail_theta >= 1e300) ? h->nunits : 0;
    h->bound = true;
    build_groups(h);
    rc = build_tiles(h, 0, default_shape(h, 0));
    if (rc == GF_OK) rc = build_tiles(h, 1, default_shape(h, 1));
    if (rc == GF_OK) rc = build_tiles(h, 2, default_shape(h, 2));
    if (rc) {
        h->bound = false;
        return rc;
    }
    return GF_OK;
}

static int transfer(gf_handle h, int32_t inst, double *links, int32_t t0, int32_t nt, int on_device, int dir,
                    int flags) {
    int rc = check_bound(h);
    if (rc) return rc;
    rc = check_inst(h, inst);
    if (rc) return rc;
    if (!links) return fail(h, GF_E_INVALID, "links is NULL");
    const InstHost &I = h->inst[inst];
    if (t0 < 0 || nt < 0 || t0 + nt > I.n[0]) return fail(h, GF_E_INVALID, "time slab [%d, %d) out of range", t0, t0 + nt);
    HIPCHK(h, hipSetDevice(h->dev));
    const int64_t Vs = I.V / I.n[0];
    const int64_t s0 = (int64_t)t0 * Vs, ns = (int64_t)nt * Vs;
    const gfs::InstDev d = inst_dev(I);
    const int st = st_code(h);
    const int reun = (flags & GF_DL_REUNITARISE) ? 1 : 0;
    if (on_device) {
        if (dir == 0)
            HIPCHK(h, gfl::convert_in(st, h->ws, d, links, s0, ns, h->stream));
        else
            HIPCHK(h, gfl::convert_out(st, h->ws, d, links, s0, ns, reun, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        return GF_OK;
    }
    const int64_t sr = site_reals(h), sb = 8 * sr;
    const int64_t per = std::max<int64_t>(1, (int64_t)(h->stage_bytes / sb));
    double *stage = wsp<double>(h, h->off_stage);
    for (int64_t s = 0; s < ns; s += per) {
        const int64_t c = std::min(per, ns - s);
        if (dir == 0) {
            HIPCHK(h, hipMemcpyAsync(stage, links + s * sr, (size_t)(c * sb), hipMemcpyHostToDevice, h->stream));
            HIPCHK(h, gfl::convert_in(st, h->ws, d, stage, s0 + s, c, h->stream));
        } else {
            HIPCHK(h, gfl::convert_out(st, h->ws, d, stage, s0 + s, c, reun, h->stream));
            HIPCHK(h, hipMemcpyAsync(links + s * sr, stage, (size_t)(c * sb), hipMemcpyDeviceToHost, h->stream));
        }
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    return GF_OK;
}

int gf_upload(gf_handle h, int32_t inst, const double *links, int32_t t0, int32_t nt, int on_device) {
    return transfer(h, inst, const_cast<double *>(links), t0, nt, on_device, 0, 0);
}

int gf_download(gf_handle h, int32_t inst, double *links, int32_t t0, int32_t nt, int on_device, int flags) {
    return transfer(h, inst, links, t0, nt, on_device, 1, flags);
}

int gf_set_overrelax(gf_handle h, double omega) {
    if (!h) return GF_E_INVALID;
    if (!(omega >= 1.0 && omega < 2.0)) return fail(h, GF_E_INVALID, "omega %g not in [1, 2)", omega);
    h->omega = omega;
    h->graph.clear();
    return GF_OK;
}

int gf_set_stochastic(gf_handle h, double p) {
    if (!h) return GF_E_INVALID;
    if (!(p >= 0.0 && p <= 1.0)) return fail(h, GF_E_INVALID, "probability %g not in [0, 1]", p);
    h->p_sr = p;
    h->graph.clear();
    return GF_OK;
}

int gf_set_seed(gf_handle h, uint64_t seed) {
    if (!h) return GF_E_INVALID;
    h->seed = seed;
    h->graph.clear();
    return GF_OK;
}

int gf_set_temperature(gf_handle h, double T) {
    if (!h) return GF_E_INVALID;
    if (!(T > 0.0) || !std::isfinite(T)) return fail(h, GF_E_INVALID, "temperature %g must be > 0", T);
    h->T = T;
    h->graph.clear();
    return GF_OK;
}

int gf_set_anneal(gf_handle h, double T0, double T1, int32_t nsteps, int32_t nmicro, uint64_t seed) {
    if (!h) return GF_E_INVALID;
    if (!(T0 > 0.0) || !(T1 > 0.0) || !std::isfinite(T0) || !std::isfinite(T1))
        return fail(h, GF_E_INVALID, "temperatures must be > 0");
    if (nsteps < 1 || nmicro < 0) return fail(h, GF_E_INVALID, "nsteps >= 1 and nmicro >= 0 required");
    h->sa_T0 = T0;
    h->sa_T1 = T1;
    h->sa_steps = nsteps;
    h->sa_micro = nmicro;
    h->seed = seed;
    h->graph.clear();
    return GF_OK;
}

int gf_sweep(gf_handle h, int update, int32_t max_sweeps, double theta_tol, int32_t check_every, int32_t *sweeps_done) {
    int rc = check_bound(h);
    if (rc) return rc;
    HIPCHK(h, hipSetDevice(h->dev));
    HIPCHK(h, gfl::fill_i32(wsp<int32_t>(h, h->off_sweeps), 0, h->nunits, h->stream));
    HIPCHK(h, gfl::fill_i32(wsp<int32_t>(h, h->off_active), 1, h->nunits, h->stream));
    if (update == GF_ANNEAL) {
        if (h->sa_steps < 1) return fail(h, GF_E_STATE, "no annealing schedule (gf_set_anneal)");
        for (int k = 0; k < h->sa_steps; ++k) {
            const double T =
                (h->sa_steps > 1) ? h->sa_T0 + (h->sa_T1 - h->sa_T0) * (double)k / (double)(h->sa_steps - 1) : h->sa_T0;
            rc = launch_sweep(h, gfs::UPD_HEATBATH, T, false, false, 0);
            if (rc) return rc;
            for (int m = 0; m < h->sa_micro; ++m) {
                rc = launch_sweep(h, gfs::UPD_MICRO, T, false, false, 1 + m);
                if (rc) return rc;
            }
            rc = count_chunk(h, 1 + h->sa_micro);
            if (rc) return rc;
        }
        rc = coulomb_finish(h);
        if (rc) return rc;
        rc = drain_timing(h);
        if (rc) return rc;
        rc = fetch_sweeps_done(h, sweeps_done);
        if (rc) return rc;
        HIPCHK(h, hipStreamSynchronize(h->stream));
        return GF_OK;
    }
    const int upd = upd_code(update);
    if (upd < 0) return fail(h, GF_E_INVALID, "bad update type %d", update);
    if (max_sweeps < 0) return fail(h, GF_E_INVALID, "max_sweeps < 0");
    if (check_every < 1) check_every = 1;
    // Checks at k = 0, c, 2c, ... measure theta and stop units on the device
    // (a check reads only the units still active; a stopped unit's partial
    // sums from its stopping check stand, since its links do not change).
    // The next chunk of sweeps is enqueued before the host reads a check's
    // status: sweep kernels skip stopped units, so a chunk queued after the
    // last unit stopped changes nothing, and the GPU never idles while the
    // host waits.  Kernel variants (FP32 / FP64 update) follow the status of
    // the check before, which keeps the schedule deterministic.
    for (int e = 0; e < 2; ++e)
        if (!h->chk_ev[e]) HIPCHK(h, hipEventCreateWithFlags(&h->chk_ev[e], hipEventDisableTiming));
    // each check also reads the per-unit active flags: groups whose units
    // have all stopped are skipped from then on, and groups with some
    // stopped units are launched in the linear tile order
    const int ng = ngroups(h);
    struct LiveGuard {
        gf_ctx *h;
        ~LiveGuard() { h->grp_live.clear(); }
    } live_guard{h};
    if (!h->hact)
        HIPCHK(h, hipHostMalloc(reinterpret_cast<void **>(&h->hact), 2 * sizeof(int32_t) * h->nunits,
                                hipHostMallocDefault));
    h->grp_live.assign(ng, 2);
    struct Pend {
        int slot, k;
    };
    Pend pend[2];
    int npend = 0, slot = 0;
    auto enqueue_check = [&](int kk) -> int {
        int r = launch_measure(h, 0, true, theta_tol, true);
        if (r) return r;
        HIPCHK(h, hipMemcpyAsync(h->hstat + 4 * slot, h->ws + h->off_status, 3 * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->hact + (size_t)slot * h->nunits, h->ws + h->off_active,
                                 sizeof(int32_t) * h->nunits, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipEventRecord(h->chk_ev[slot], h->stream));
        pend[npend++] = {slot, kk};
        slot ^= 1;
        return GF_OK;
    };
    int k = 0;
    bool stopped = false;
    // sweeps from k until every unit stopped (stopped = true) or max_sweeps
    auto run_until_stopped = [&]() -> int {
        for (;;) {
            if (npend == 2 || (k >= max_sweeps && npend > 0)) {
                const Pend c = pend[0];
                pend[0] = pend[1];
                --npend;
                HIPCHK(h, hipEventSynchronize(h->chk_ev[c.slot]));
                const int32_t *st = h->hstat + 4 * c.slot;
                if (st[1] != 0) {
                    HIPCHK(h, hipStreamSynchronize(h->stream));
                    (void)fetch_sweeps_done(h, sweeps_done);
                    return fail(h, GF_E_NONFINITE, "F or theta not finite in %d unit(s) after %d sweeps", st[1],
                                c.k);
                }
                h->n_active = st[0];
                h->n_tail = st[2];
                if (st[0] == 0) {
                    stopped = true;
                    return GF_OK;
                }
                set_live_groups(h, h->hact + (size_t)c.slot * h->nunits);
                continue;
            }
            if (k >= max_sweeps) return GF_OK;
            const int n = std::min(check_every - k % check_every, max_sweeps - k);
            int r = run_sweeps(h, upd, n, k, n == check_every);
            if (r) return r;
            k += n;
            if (k % check_every == 0) {
                r = enqueue_check(k);
                if (r) return r;
            }
        }
    };
    rc = enqueue_check(0);
    if (rc) return rc;
    rc = run_until_stopped();
    if (rc) return rc;
    // FP32 storages with reprojection in use deliver their links reprojected
    // in FP64 (Sec. 4.5), and the reprojection rounded back to FP32 moves
    // theta slightly: so the units that stopped are reprojected and checked
    // again, and those whose theta is no longer below the tolerance continue
    // (chunks of check_every sweeps, within max_sweeps) until a check on
    // reprojected links passes.
    const bool fp32_store = (h->storage == GF_MIXED_F32_R12 || h->storage == GF_F32_R12);
    if (stopped && fp32_store && h->reunit_every > 0) {
        std::vector<int32_t> ran(h->nunits, 1);  // first pass: every unit
        for (;;) {
            HIPCHK(h, hipStreamSynchronize(h->stream));  // queued chunks and checks have run
            npend = 0;
            for (int u = 0; u < h->nunits;) {
                if (!ran[u]) {
                    ++u;
                    continue;
                }
                int v = u;
                while (v < h->nunits && ran[v]) ++v;
                rc = launch_reunit_units(h, false, u, v);
                if (rc) return rc;
                u = v;
            }
            HIPCHK(h, hipMemcpyAsync(h->ws + h->off_active, ran.data(), sizeof(int32_t) * h->nunits,
                                     hipMemcpyHostToDevice, h->stream));
            rc = launch_measure(h, 0, true, theta_tol, true);
            if (rc) return rc;
            HIPCHK(h, hipMemcpyAsync(h->hstat, h->ws + h->off_status, 3 * sizeof(int32_t), hipMemcpyDeviceToHost,
                                     h->stream));
            HIPCHK(h, hipMemcpyAsync(ran.data(), h->ws + h->off_active, sizeof(int32_t) * h->nunits,
                                     hipMemcpyDeviceToHost, h->stream));
            HIPCHK(h, hipStreamSynchronize(h->stream));
            if (h->hstat[1] != 0) {
                (void)fetch_sweeps_done(h, sweeps_done);
                return fail(h, GF_E_NONFINITE, "F or theta not finite in %d unit(s) after reprojection", h->hstat[1]);
            }
            h->n_active = h->hstat[0];
            h->n_tail = h->hstat[2];
            if (h->n_active == 0) break;
            set_live_groups(h, ran.data());
            if (k >= max_sweeps) {
                stopped = false;
                break;
            }
            // k is a multiple of check_every here (a chunk ends at one, or
            // at max_sweeps), so the chunks keep their graph patterns
            stopped = false;
            rc = run_until_stopped();
            if (rc) return rc;
            if (!stopped) break;
        }
    }
    int status = stopped ? GF_OK : GF_NOT_CONVERGED;
    rc = coulomb_finish(h);
    if (rc) return rc;
    rc = drain_timing(h);
    if (rc) return rc;
    rc = fetch_sweeps_done(h, sweeps_done);
    if (rc) return rc;
    if (status == GF_NOT_CONVERGED) (void)fail(h, GF_NOT_CONVERGED, "not converged after %d sweeps", max_sweeps);
    return status;
}

int gf_halfsweep(gf_handle h, int update, int parity) {
    int rc = check_bound(h);
    if (rc) return rc;
    const int upd = upd_code(update);
    if (upd < 0) return fail(h, GF_E_INVALID, "bad update type %d", update);
    if (parity != 0 && parity != 1) return fail(h, GF_E_INVALID, "parity must be 0 or 1");
    HIPCHK(h, hipSetDevice(h->dev));
    HIPCHK(h, gfl::fill_i32(wsp<int32_t>(h, h->off_active), 1, h->nunits, h->stream));
    rc = launch_half(h, upd, parity, h->T, false, 0);
    if (rc) return rc;
    rc = drain_timing(h);
    if (rc) return rc;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return GF_OK;
}

static int measure_units(gf_handle h, int with_unitarity) {
    int rc = check_bound(h);
    if (rc) return rc;
    HIPCHK(h, hipSetDevice(h->dev));
    rc = launch_measure(h, with_unitarity);
    if (rc) return rc;
    HIPCHK(h, hipMemcpyAsync(h->hres, h->ws + h->off_res, sizeof(double) * 4 * h->nunits, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return GF_OK;
}

int gf_measure(gf_handle h, int32_t inst, double *F, double *theta) {
    int rc = check_bound(h);
    if (rc) return rc;
    rc = check_inst(h, inst);
    if (rc) return rc;
    rc = measure_units(h, 0);
    if (rc) return rc;
    const InstHost &I = h->inst[inst];
    double f = 0.0, t = 0.0;
    for (int u = I.unit0; u < I.unit0 + I.nunits; ++u) {
        f += h->hres[4 * u];
        t += h->hres[4 * u + 1];
    }
    f /= I.nunits;
    t /= I.nunits;
    if (F) *F = f;
    if (theta) *theta = t;
    if (!std::isfinite(f) || !std::isfinite(t)) return fail(h, GF_E_NONFINITE, "F or theta not finite");
    return GF_OK;
}

int gf_measure_timeslices(gf_handle h, int32_t inst, double *F_t, double *theta_t) {
    int rc = check_bound(h);
    if (rc) return rc;
    rc = check_inst(h, inst);
    if (rc) return rc;
    if (h->gauge != GF_COULOMB) return fail(h, GF_E_STATE, "per time-slice values need Coulomb gauge");
    rc = measure_units(h, 0);
    if (rc) return rc;
    const InstHost &I = h->inst[inst];
    bool fin = true;
    for (int k = 0; k < I.nunits; ++k) {
        const double f = h->hres[4 * (I.unit0 + k)], t = h->hres[4 * (I.unit0 + k) + 1];
        if (F_t) F_t[k] = f;
        if (theta_t) theta_t[k] = t;
        fin = fin && std::isfinite(f) && std::isfinite(t);
    }
    if (!fin) return fail(h, GF_E_NONFINITE, "F or theta not finite");
    return GF_OK;
}

int gf_unitarity(gf_handle h, int32_t inst, double *mean, double *maxv) {
    int rc = check_bound(h);
    if (rc) return rc;
    rc = check_inst(h, inst);
    if (rc) return rc;
    rc = measure_units(h, 1);
    if (rc) return rc;
    const InstHost &I = h->inst[inst];
    double s = 0.0, m = 0.0;
    for (int u = I.unit0; u < I.unit0 + I.nunits; ++u) {
        s += h->hres[4 * u + 2];
        m = std::max(m, h->hres[4 * u + 3]);
    }
    if (mean) *mean = s / I.nunits;
    if (maxv) *maxv = m;
    return GF_OK;
}

int gf_reunitarise(gf_handle h) {
    int rc = check_bound(h);
    if (rc) return rc;
    HIPCHK(h, hipSetDevice(h->dev));
    rc = launch_reunit_all(h, false);
    if (rc) return rc;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return GF_OK;
}

int gf_get_sweep_index(gf_handle h, int32_t inst, uint64_t *index) {
    int rc = check_bound(h);
    if (rc) return rc;
    rc = check_inst(h, inst);
    if (rc) return rc;
    if (!index) return fail(h, GF_E_INVALID, "index is NULL");
    HIPCHK(h, hipMemcpyAsync(index, h->ws + h->off_sweepix + sizeof(uint64_t) * inst, sizeof(uint64_t),
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return GF_OK;
}

int gf_set_sweep_index(gf_handle h, int32_t inst, uint64_t index) {
    int rc = check_bound(h);
    if (rc) return rc;
    rc = check_inst(h, inst);
    if (rc) return rc;
    uint64_t v = index;
    HIPCHK(h, hipMemcpyAsync(h->ws + h->off_sweepix + sizeof(uint64_t) * inst, &v, sizeof(uint64_t),
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return GF_OK;
}

// compute precisions of the update this configuration uses (bit 0 FP32, bit 1 FP64)
static int used_precisions(const gf_ctx *h) {
    if (h->storage == GF_F32_R12) return 1;
    if (h->storage != GF_MIXED_F32_R12) return 2;
    if (h->tail_theta <= 0.0) return 1;
    if (h->tail_theta >= 1e300) return 2;
    return 3;
}

// the precision doing most of the sweeps
static int dominant_ctd(const gf_ctx *h) { return (used_precisions(h) & 1) ? 0 : 1; }

static int check_table(gf_ctx *h, int kernels) {
    if (kernels < GF_KERNELS_FP32 || kernels > GF_KERNELS_HEATBATH)
        return fail(h, GF_E_INVALID, "kernel table %d (GF_KERNELS_FP32, _FP64 or _HEATBATH)", kernels);
    return GF_OK;
}

int gf_set_launch(gf_handle h, int lanes_per_site, int block) {
    int rc = check_bound(h);
    if (rc) return rc;
    if (block != 0 && gfl::block_index(block) < 0) return fail(h, GF_E_INVALID, "block %d not available", block);
    int set = 0;
    for (int tab = 0; tab < 3; ++tab) {
        Shape sh;
        sh.W = lanes_per_site == 0 ? default_shape(h, tab).W : lanes_per_site;
        sh.B = block == 0 ? 256 : block;
        if (!table_kernel(h, tab, sh)) continue;
        rc = build_tiles(h, tab, sh);
        if (rc) return rc;
        ++set;
    }
    if (!set)
        return fail(h, GF_E_INVALID, "no variant with %d wavefronts per site group and %d threads per block",
                    lanes_per_site, block);
    return GF_OK;
}

int gf_set_shape(gf_handle h, int kernels, int waves_per_site, int block, int flags) {
    int rc = check_bound(h);
    if (rc) return rc;
    rc = check_table(h, kernels);
    if (rc) return rc;
    if (flags & ~(GF_SHAPE_NONTEMPORAL | GF_SHAPE_LINEAR_TILES)) return fail(h, GF_E_INVALID, "flags %d", flags);
    Shape sh;
    sh.W = waves_per_site;
    sh.B = block;
    sh.nt = (flags & GF_SHAPE_NONTEMPORAL) ? 1 : 0;
    sh.xcd = (flags & GF_SHAPE_LINEAR_TILES) ? 0 : 1;
    if (!table_kernel(h, kernels, sh))
        return fail(h, GF_E_INVALID, "no variant of kernel table %d with W %d, B %d, flags %d", kernels,
                    waves_per_site, block, flags);
    return build_tiles(h, kernels, sh);
}

int gf_get_shape(gf_handle h, int kernels, int *waves_per_site, int *block, int *flags) {
    int rc = check_bound(h);
    if (rc) return rc;
    rc = check_table(h, kernels);
    if (rc) return rc;
    const Shape &sh = h->shape[kernels];
    if (waves_per_site) *waves_per_site = sh.W;
    if (block) *block = sh.B;
    if (flags) *flags = (sh.nt ? GF_SHAPE_NONTEMPORAL : 0) | (sh.xcd ? 0 : GF_SHAPE_LINEAR_TILES);
    return GF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- autotuning
namespace {

// what a tuning key holds: device architecture, gauge group, gauge, storage,
// kernel table, and the size class of the bound configuration (half-sites
// and units, each rounded to a power of two)
std::string tune_key(gf_ctx *h, int tab) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, h->dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch = arch.substr(0, c);
    }
    int64_t hs = 0;
    for (const auto &u : h->units) hs += u.n;
    char buf[256];
    snprintf(buf, sizeof buf, "%s/su%d/gauge%d/storage%d/kernels%d/halfsites2^%ld/units2^%ld", arch.c_str(), h->nc,
             h->gauge, h->storage, tab, std::lround(std::log2((double)std::max<int64_t>(hs, 1))),
             std::lround(std::log2((double)std::max(h->nunits, 1))));
    return buf;
}

int load_tune_cache(gf_ctx *h) {
    h->tune_cache.clear();
    std::ifstream f(h->tune_path);
    if (!f) return GF_OK;  // no file yet
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        Shape sh;
        if (!(is >> key >> sh.W >> sh.B >> sh.nt >> sh.xcd)) continue;
        if (gfl::wave_index(sh.W) < 0 || gfl::block_index(sh.B) < 0 || (sh.nt & ~1) || (sh.xcd & ~1)) continue;
        h->tune_cache[key] = sh;
    }
    return GF_OK;
}

int save_tune_cache(gf_ctx *h) {
    const std::string tmp = h->tune_path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return fail(h, GF_E_INVALID, "cannot write the tuning cache %s", tmp.c_str());
        for (const auto &kv : h->tune_cache)
            f << kv.first << ' ' << kv.second.W << ' ' << kv.second.B << ' ' << kv.second.nt << ' ' << kv.second.xcd
              << '\n';
        if (!f) return fail(h, GF_E_INVALID, "cannot write the tuning cache %s", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), h->tune_path.c_str()) != 0)
        return fail(h, GF_E_INVALID, "cannot replace the tuning cache %s", h->tune_path.c_str());
    return GF_OK;
}

// The state trial sweeps change: the link planes and Coulomb accumulators
// (workspace [0, off_inst)) and the per-unit results, stop and tail flags,
// sweep counts and sweep indices ([off_res, off_status + 256)).  Saved to
// host memory and written back, so tuning leaves the caller's state as it
// was.
struct Snapshot {
    std::vector<char> lat, book;
    int n_active = 0, n_tail = 0;
};

int save_state(gf_ctx *h, Snapshot &sn) {
    try {
        sn.lat.resize(h->off_inst);
        sn.book.resize(h->off_status + 256 - h->off_res);
    } catch (const std::bad_alloc &) {
        return fail(h, GF_E_NOMEM, "autotuning: no host memory for the %zu bytes of saved state",
                    (size_t)h->off_inst);
    }
    HIPCHK(h, hipMemcpyAsync(sn.lat.data(), h->ws, sn.lat.size(), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(sn.book.data(), h->ws + h->off_res, sn.book.size(), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    sn.n_active = h->n_active;
    sn.n_tail = h->n_tail;
    return GF_OK;
}

int restore_state(gf_ctx *h, const Snapshot &sn) {
    HIPCHK(h, hipMemcpyAsync(h->ws, sn.lat.data(), sn.lat.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->ws + h->off_res, sn.book.data(), sn.book.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->n_active = sn.n_active;
    h->n_tail = sn.n_tail;
    return GF_OK;
}

// One visit of shape `sh`: switch to it, run one untimed sweep, then time
// `sweeps` back-to-back sweeps between two events, group by group as
// gf_sweep runs them (the figure includes launch gaps); ms per sweep.
int visit_shape(gf_ctx *h, int tab, int upd, const Shape &sh, int sweeps, hipEvent_t e0, hipEvent_t e1,
                float *ms_per_sweep) {
    int rc = build_tiles(h, tab, sh);
    if (rc == GF_OK) rc = enqueue_chunk(h, upd, 1, 0, false);
    if (rc == GF_OK) rc = count_chunk(h, 1);
    if (rc) return rc;
    HIPCHK(h, hipEventRecord(e0, h->cur));
    rc = enqueue_chunk(h, upd, sweeps, 0, false);
    if (rc == GF_OK) rc = count_chunk(h, sweeps);
    if (rc) return rc;
    HIPCHK(h, hipEventRecord(e1, h->cur));
    HIPCHK(h, hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
    *ms_per_sweep = ms / sweeps;
    return GF_OK;
}

float median_of(std::vector<float> t) {
    std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
    return t[t.size() / 2];
}

// Time every shape of table `tab` with update `upd` and keep the fastest, in
// two stages, after a warm-up: untimed sweeps for about 20 ms, since the
// first milliseconds of work after an idle GPU (the host copy of the saved
// state just before) run at lower clocks and would count against the shapes
// visited first.  Screening: `reps` rounds of a short visit (3 timed sweeps) to
// every shape.  Final: the kFinal shapes with the smallest screening medians
// get max(reps, 3) rounds of long visits (12 timed sweeps); the smallest
// median of those wins.  Shapes of large lattices lie within a few per cent
// of each other and some of them vary more from visit to visit than that, so
// a short screening alone can crown one whose lucky visits it saw.  Rounds
// interleave the shapes (drifts of clock or temperature hit all of them
// alike).  All units are active during the trial.
int time_shapes(gf_ctx *h, int tab, int upd, int reps, hipEvent_t e0, hipEvent_t e1, Shape *best) {
    constexpr int kScreen = 3, kLong = 12, kFinal = 4;
    const std::vector<Shape> cand = table_shapes(h, tab);
    if (cand.empty()) return fail(h, GF_E_INVALID, "kernel table %d has no variant", tab);
    HIPCHK(h, gfl::fill_i32(wsp<int32_t>(h, h->off_active), 1, h->nunits, h->stream));
    h->n_active = h->nunits;
    {
        float ms = 0.f;
        int rc = visit_shape(h, tab, upd, cand[0], 1, e0, e1, &ms);
        const int nwarm = std::max(1, std::min(256, (int)std::ceil(20.0f / std::max(ms, 1e-3f))));
        if (rc == GF_OK) rc = enqueue_chunk(h, upd, nwarm, 0, false);
        if (rc == GF_OK) rc = count_chunk(h, nwarm);
        if (rc) return rc;
    }
    std::vector<std::vector<float>> times(cand.size());
    for (int r = 0; r < reps; ++r)
        for (size_t k = 0; k < cand.size(); ++k) {
            float ms = 0.f;
            const int rc = visit_shape(h, tab, upd, cand[k], kScreen, e0, e1, &ms);
            if (rc) return rc;
            times[k].push_back(ms);
        }
    std::vector<std::pair<float, size_t>> order;
    for (size_t k = 0; k < cand.size(); ++k) order.push_back({median_of(times[k]), k});
    std::sort(order.begin(), order.end());
    order.resize(std::min(order.size(), (size_t)kFinal));
    *best = cand[order[0].second];
    if (order.size() == 1) return GF_OK;
    std::vector<std::vector<float>> fin(order.size());
    for (int r = 0; r < std::max(reps, 3); ++r)
        for (size_t i = 0; i < order.size(); ++i) {
            float ms = 0.f;
            const int rc = visit_shape(h, tab, upd, cand[order[i].second], kLong, e0, e1, &ms);
            if (rc) return rc;
            fin[i].push_back(ms);
        }
    float bt = 3.4e38f;
    for (size_t i = 0; i < order.size(); ++i) {
        const float med = median_of(fin[i]);
        if (med < bt) {
            bt = med;
            *best = cand[order[i].second];
        }
    }
    return GF_OK;
}

// tune tables `tabs` (with update upd), from the cache where it has them
int autotune_tables(gf_ctx *h, const std::vector<int> &tabs, int upd, int reps) {
    if (reps < 1) reps = 1;
    int rc = drain_timing(h);
    if (rc) return rc;
    std::vector<int> todo;
    for (int tab : tabs) {
        auto it = h->tune_path.empty() ? h->tune_cache.end() : h->tune_cache.find(tune_key(h, tab));
        if (it != h->tune_cache.end() && table_kernel(h, tab, it->second)) {
            rc = build_tiles(h, tab, it->second);
            if (rc) return rc;
        } else {
            todo.push_back(tab);
        }
    }
    if (todo.empty()) return GF_OK;
    hipEvent_t e0 = take_event(h), e1 = take_event(h);
    if (!e0 || !e1) return fail(h, GF_E_HIP, "hipEventCreate failed");
    // trial sweeps are plain launches without reprojection or per-launch
    // events; the caller's settings and the events come back on every path
    struct Restore {
        gf_ctx *h;
        bool timing;
        int reunit_every;
        hipEvent_t e0, e1;
        ~Restore() {
            h->timing = timing;
            h->reunit_every = reunit_every;
            h->force_ctd = -1;
            h->ev_pool.push_back(e0);
            h->ev_pool.push_back(e1);
        }
    } restore{h, h->timing, h->reunit_every, e0, e1};
    h->timing = false;
    h->reunit_every = 0;
    Snapshot sn;
    rc = save_state(h, sn);
    if (rc) return rc;
    std::vector<Shape> best(todo.size());
    for (size_t i = 0; i < todo.size() && rc == GF_OK; ++i) {
        h->force_ctd = (upd == gfs::UPD_HEATBATH) ? -1 : todo[i];
        rc = time_shapes(h, todo[i], upd, reps, e0, e1, &best[i]);
        h->force_ctd = -1;
    }
    const int rs = restore_state(h, sn);
    if (rc) return rc;
    if (rs) return rs;
    for (size_t i = 0; i < todo.size(); ++i) {
        rc = build_tiles(h, todo[i], best[i]);
        if (rc) return rc;
        if (!h->tune_path.empty()) h->tune_cache[tune_key(h, todo[i])] = best[i];
    }
    if (!h->tune_path.empty()) return save_tune_cache(h);
    return GF_OK;
}

}  // namespace

extern "C" {

int gf_autotune(gf_handle h, int reps, int *lanes_per_site, int *block) {
    int rc = check_bound(h);
    if (rc) return rc;
    const int used = used_precisions(h);
    std::vector<int> tabs;
    for (int ctd = 0; ctd < 2; ++ctd)
        if (used & (1 << ctd)) tabs.push_back(ctd);
    rc = autotune_tables(h, tabs, gfs::UPD_OR, reps);
    if (rc) return rc;
    if (lanes_per_site) *lanes_per_site = h->shape[dominant_ctd(h)].W;
    if (block) *block = h->shape[dominant_ctd(h)].B;
    return GF_OK;
}

int gf_autotune_heatbath(gf_handle h, int reps, int *lanes_per_site, int *block) {
    int rc = check_bound(h);
    if (rc) return rc;
    rc = autotune_tables(h, {2}, gfs::UPD_HEATBATH, reps);
    if (rc) return rc;
    if (lanes_per_site) *lanes_per_site = h->shape[2].W;
    if (block) *block = h->shape[2].B;
    return GF_OK;
}

int gf_set_tune_cache(gf_handle h, const char *path) {
    if (!h) return GF_E_INVALID;
    h->tune_path = path ? path : "";
    if (h->tune_path.empty()) {
        h->tune_cache.clear();
        return GF_OK;
    }
    return load_tune_cache(h);
}

int gf_set_timing(gf_handle h, int every) {
    if (!h) return GF_E_INVALID;
    if (every < 0) return fail(h, GF_E_INVALID, "timing interval < 0");
    int rc = drain_timing(h);
    if (rc) return rc;
    h->timing = every != 0;
    h->time_every = every > 0 ? every : 1;
    h->chunk_seq = 0;
    h->t_sum_ms[0] = h->t_sum_ms[1] = 0.0;
    h->t_count[0] = h->t_count[1] = 0;
    return GF_OK;
}

int gf_kernel_time(gf_handle h, int which, int64_t *launches, double *mean_ms) {
    if (!h) return GF_E_INVALID;
    if (which < 0 || which > 2) return fail(h, GF_E_INVALID, "which must be 0, 1 or 2");
    int rc = drain_timing(h);
    if (rc) return rc;
    int64_t n = 0;
    double ms = 0.0;
    if (which == 0 || which == 1) {
        n += h->t_count[0];
        ms += h->t_sum_ms[0];
    }
    if (which == 0 || which == 2) {
        n += h->t_count[1];
        ms += h->t_sum_ms[1];
    }
    if (launches) *launches = n;
    if (mean_ms) *mean_ms = n ? ms / (double)n : 0.0;
    return GF_OK;
}

int gf_set_cache_budget(gf_handle h, int64_t bytes) {
    if (!h) return GF_E_INVALID;
    if (bytes < 0) return fail(h, GF_E_INVALID, "cache budget < 0");
    h->cache_budget = bytes;
    if (h->bound) {
        build_groups(h);
        h->graph.clear();
    }
    return GF_OK;
}

int gf_cache_groups(gf_handle h, int32_t *groups) {
    if (!h) return GF_E_INVALID;
    int rc = check_bound(h);
    if (rc) return rc;
    if (groups) *groups = ngroups(h);
    return GF_OK;
}

int gf_set_graph(gf_handle h, int enable) {
    if (!h) return GF_E_INVALID;
    h->use_graph = enable != 0;
    h->graph.clear();
    return GF_OK;
}


int gf_measure_noalloc(int hip_device, void *hip_stream, int gauge, const int32_t dims[4], const double *links,
                       double *out) {
    if (!dims || !links || !out) return fail(nullptr, GF_E_INVALID, "gf_measure_noalloc: dims, links or out is NULL");
    if (gauge != GF_LANDAU && gauge != GF_COULOMB && gauge != GF_MAG)
        return fail(nullptr, GF_E_INVALID, "gf_measure_noalloc: unknown gauge %d", gauge);
    int64_t V = 1;
    for (int k = 0; k < 4; ++k) {
        if (dims[k] < 2 || (dims[k] & 1))
            return fail(nullptr, GF_E_DIMS, "gf_measure_noalloc: extent %d of dimension %d is not even and >= 2",
                        dims[k], k);
        V *= dims[k];
        if (V > GF_NOALLOC_MAX_SITES)
            return fail(nullptr, GF_E_DIMS, "gf_measure_noalloc: lattice larger than %lld sites",
                        (long long)GF_NOALLOC_MAX_SITES);
    }
    int ndev = 0, prev = -1;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return fail(nullptr, GF_E_HIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (hip_device < 0 || hip_device >= ndev)
        return fail(nullptr, GF_E_INVALID, "gf_measure_noalloc: no HIP device %d", hip_device);
    e = hipGetDevice(&prev);
    if (e != hipSuccess) return fail(nullptr, GF_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (prev != hip_device) {
        e = hipSetDevice(hip_device);
        if (e != hipSuccess) return fail(nullptr, GF_E_HIP, "hipSetDevice: %s", hipGetErrorString(e));
    }
    double *scr = nullptr;
    e = gfl::noalloc_scratch(hip_device, &scr, nullptr);
    if (e == hipSuccess) e = gfl::measure_nat(gauge, links, dims, out, scr, reinterpret_cast<hipStream_t>(hip_stream));
    if (prev != hip_device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail(nullptr, GF_E_HIP, "gf_measure_noalloc: %s", hipGetErrorString(e));
    return GF_OK;
}

}  // extern "C"
