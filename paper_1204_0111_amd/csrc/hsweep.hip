// Context and C-ABI entry points of the sweeping preconditioner.
//
// Setup (Sec. 1.1, Alg. 1.4) factors every panel of every problem; the
// fronts of one elimination-tree depth over all panels and problems share
// each launch (Sec. 2: panel factorisations are independent).  The sweep
// (Alg. 1.5) runs the panel solves in order (they are sequential), all
// right-hand sides of a problem together.  GMRES(k) (Sec. 2.4) is flexible
// and right-preconditioned, in FP64 on the device; the host reads one
// residual estimate per Arnoldi step to decide when to stop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "devtypes.hpp"
#include "hsweep.h"
#include "kernels.hpp"
#include "plan.hpp"

using namespace hsw;

namespace {

std::string g_create_error;

struct Launch {
    int64_t off;
    int count;
    int k;
    double bytes_per_esz = 0;  // algorithmic bytes of the launch / bytes per complex entry
    double cmac = 0;           // algorithmic complex multiply-adds
};

struct DepthSchedule {
    Launch assemble;
    std::vector<Launch> ldlt, panel, trail;  // one per pivot block
    // left-looking alternative: update of block column k before its pivots
    // are factored (empty launch for k = 0), and one final Schur update of F_BR
    std::vector<Launch> left;
    Launch schur;
    // hybrid: the right-looking update restricted to the pivot columns,
    // with F_BR left to the final Schur update
    std::vector<Launch> pivots;
    int nfronts = 0;
};

// Right-hand-side groups that are tuned separately: 1, 2, 3-4, 5+ columns.
constexpr int N_RHS_KEYS = 4;
inline int rhs_key(int nrhs) { return nrhs <= 1 ? 0 : nrhs <= 2 ? 1 : nrhs <= 4 ? 2 : 3; }

// Selection of the triangular passes with the kept factors in a level's
// fsel / bsel, past the block shapes of the inverse passes.
constexpr int TRI_F = N_FWD_SHAPES, TRI_B = N_BWD_SHAPES;

struct SolveLevel {
    // work items of every block shape (plan.hpp) of the two passes
    int64_t foff[N_FWD_SHAPES] = {}, boff[N_BWD_SHAPES] = {};
    int fcount[N_FWD_SHAPES] = {}, bcount[N_BWD_SHAPES] = {};
    int fsel[N_RHS_KEYS] = {}, bsel[N_RHS_KEYS] = {};  // shape in use, per right-hand-side group
    // one work item per front for the triangular passes (selected as shape
    // TRI_F / TRI_B)
    int64_t toff = 0;
    int tcount = 0;
    int smax = 0, nmax = 0;
    // matrix-core passes: items of 64 rows / columns (0) or of 16 (1) per
    // pass, picked by the autotuner; -1: the fixed rule
    int mm_f = -1, mm_b = -1;
    // algorithmic traffic, for a panel whose own planes start at plane p
    // (p = 0..nz): the G entries a pass needs (also its complex multiply-adds
    // per right-hand side) -- those of the fronts with children, plus, for the
    // leaves, only the columns from the first pivot on plane p, since the
    // passes skip the columns of a leaf that multiply exact zeros -- and the
    // bytes per right-hand side of the vectors each pass must read and write
    double g_inner = 0;
    std::vector<double> g_leaf, fwd_vec, bwd_vec;
    double g_need(int p) const { return g_inner + g_leaf[p]; }
};

struct KernelTimer {
    std::string kernel;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    int64_t launches = 0;
    double bytes = 0, flops = 0;
};

// A sweep captured as a HIP graph, for one problem and right-hand-side count,
// operating on its own copy `z` of the vector (N_pad x nrhs).
struct SweepGraph {
    int prob = 0, nrhs = 0;
    hipGraphExec_t exec = nullptr;
    void* z = nullptr;
    int cycle_k = 0;  // > 0: the k Arnoldi steps of a GMRES cycle (device-side test), not a sweep
};

struct ProbHost {
    int N[3] = {0, 0, 0};
    int64_t Npad = 0, Nint = 0;
    int m = 0;
    int panel_base = 0;  // global panel id of panel 0
    int64_t c_off = 0;   // offset of the velocity in the context's copy
    double setup_cmac = 0, inverse_cmac = 0, apply_cmac = 0;
    int64_t factor_entries = 0;
    int levels = 0;
};

}  // namespace

// A solve lane: a stream and the workspaces of the panel solves and of GMRES
// that run on it.  Lane 0 runs on the context's stream; hsw_solve spreads the
// problems of a context over several lanes, one host thread each.
struct Lane {
    hipStream_t st = nullptr;
    void *d_xmid = nullptr, *d_xu = nullptr, *d_c2 = nullptr;  // panel-solve workspace
    int nrhs_cap = 0;
    // workspace of the matrix-core passes, [entry][16] blocks per group of 16
    // right-hand sides: each front's [x_S; -x_U], the child-contribution
    // slots of every panel class (each class its own zeroed region) and the
    // right-hand side in elimination order (likewise per class)
    void *d_mxu = nullptr, *d_mc2 = nullptr, *d_mh2 = nullptr;  // [x_S; -x_U] per front, slots, h2
    void* d_mpart = nullptr;  // partial blocks of the split-contraction forms
    int mm_groups = 0;
    std::vector<std::pair<void*, size_t>> gws;  // GMRES workspace: (pointer, bytes) per buffer
    const int* run = nullptr;  // device flag the pass kernels test (GMRES cycles with the test on the device)
};

struct hsw_ctx {
    hipStream_t st = nullptr;
    int device = 0;
    hsw_precision prec = HSW_C128;
    int esz = 16;  // bytes per complex entry of the factors
    std::vector<hsw_problem> probs;
    std::vector<ProbHost> ph;
    std::vector<LatTree> trees;
    std::vector<PanelClass> classes;
    std::vector<int> cls_perm_off, cls_ulist_off, cls_cmap_off, cls_pmap_off;
    std::vector<PanelDev> pan_h;
    std::vector<ProbDev> prob_h;
    std::vector<FrontInst> inst_h;
    std::vector<DepthSchedule> fsched;  // index = depth
    // selective inversion and the copy of L_F^{-1} over L_F: one launch each
    // over all fronts when the scratch for every L_F^{-1} fits (inv_launch,
    // lfcopy_all), else one pair per tree depth with the scratch of the
    // largest depth
    Launch inv_launch{0, 0, 0}, lfcopy_all{0, 0, 0};
    std::vector<Launch> inv_depth, lfcopy_depth;
    std::vector<int64_t> toff_all;  // scratch offsets of the one-launch layout
    int64_t inv_scratch = 0, inv_scratch_all = 0;
    bool inv_by_depth = false;
    bool full_inverse = false;  // form every column of G (else leaves skip their auxiliary-plane columns)
    bool keep_factors = false; // keep L next to G (a separate G block) instead of inverting in place
    void* d_T = nullptr;       // L_F^{-1} scratch of one depth
    std::vector<std::vector<SolveLevel>> slevels;  // per class, per depth
    int maxdepth = 0;
    int64_t ws_size[2] = {0, 0};
    int64_t L_size = 0, D_size = 0;
    int max_naux = 0;
    int64_t max_wsize = 0, max_c2 = 0;
    // per class: first entry of its region of the matrix-core passes'
    // child-contribution slots (sum of the earlier classes' c2size); the
    // right-hand-side region uses cls_perm_off
    std::vector<int64_t> cls_c2_base;
    int64_t total_c2 = 0, total_naux = 0;
    int64_t et_size = 0;
    std::vector<int64_t> et_prob_off, et_panel_off;

    // device
    FrontInst* d_inst = nullptr;
    PanelDev* d_pan = nullptr;
    ProbDev* d_prob = nullptr;
    int *d_perm = nullptr, *d_ulist = nullptr, *d_cmap = nullptr;
    int2* d_fwork = nullptr;
    int* d_pmap = nullptr;
    int* d_hmap = nullptr;
    SolveItem* d_sitems = nullptr;
    Cx<double>* d_et = nullptr;
    double* d_c = nullptr;
    void *d_L = nullptr, *d_G = nullptr, *d_dinv = nullptr, *d_ws[2] = {nullptr, nullptr};
    int* d_err = nullptr;
    // solve lanes (lane 0 on st; workspaces grown on demand)
    std::vector<Lane> lanes;
    int nlanes = 4;
    bool in_lanes = false;  // set while hsw_solve runs problems on several lanes
    std::mutex err_mu;
    bool autotune = true;
    bool tuned[N_RHS_KEYS] = {};
    bool tuned_mm = false;  // the matrix-core passes' item sizes
    // triangular passes with the kept factors: 0 never, 1 at every depth,
    // 2 where the autotuner finds them faster than the inverse passes
    int tri_mode = 2;
    // captured sweeps, their stream and the events joining it to st
    bool use_graph = false;  // measured slower than stream launches for the sweep
    int update_order = -1;   // Schur updates: -1 default (hybrid), 0 right-, 1 left-looking, 2 hybrid
    bool block_gmres = false;  // one block Krylov space per group of <= 16 right-hand sides
    bool gmres_device_test = false;  // GMRES: convergence tested on the device, one read per cycle
    bool tune_report = false;        // print the autotuner's timings (environment HSW_TUNE_REPORT=1)
    bool bf16_mfma = true;     // HSW_C64_BF16GEMM: Schur updates on the BF16 matrix cores
    // matrix-core pass forms for every depth (-1: the tuned choice; the
    // forms of launch_fwd_mm and launch_bwd_mm)
    int mm_fwd_form = -1, mm_bwd_form = -1;
    // right-hand-side count from which the solves take the matrix-core passes
    // (groups of 16, the last one padded)
    int mm_min_rhs = MM_DEFAULT_FROM;
    std::vector<SweepGraph> graphs;
    hipStream_t gst = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};

    KernelTimer timer;
    bool assembled = false, factored = false;
    double t_setup = 0;
    int bad_inst = -1, bad_pivot = -1;
    std::string err;
};

static hsw_status fail(hsw_ctx* ctx, hsw_status s, const std::string& msg) {
    std::lock_guard<std::mutex> g(ctx->err_mu);
    ctx->err = msg;
    return s;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ctx, HSW_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

hsw::LaunchTiming& hsw::launch_timing() {
    static thread_local LaunchTiming lt;
    return lt;
}

// Run `launch` (one kernel launch when count > 0); when the named class is
// being timed the launch records a pair of HIP events at its own start and end.
template <class F>
static void timed(hsw_ctx* ctx, const char* cls, int count, double bytes, double flops, F&& launch) {
    KernelTimer& t = ctx->timer;
    if (count > 0 && t.on && t.kernel == cls) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            launch();
            return;
        }
        LaunchTiming& lt = launch_timing();
        lt.start = a;
        lt.stop = b;
        launch();
        lt.start = lt.stop = nullptr;
        t.ev.emplace_back(a, b);
        t.launches += 1;
        t.bytes += bytes;
        t.flops += flops;
    } else {
        launch();
    }
}

template <typename P>
static hipError_t dalloc(P** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    return hipMalloc((void**)p, bytes);
}

static void drop_graphs(hsw_ctx* ctx) {
    for (SweepGraph& g : ctx->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.z) (void)hipFree(g.z);
    }
    ctx->graphs.clear();
}

static void free_lane(Lane& L, bool own_stream) {
    for (auto& w : L.gws)
        if (w.first) (void)hipFree(w.first);
    L.gws.clear();
    for (void** p : {&L.d_xmid, &L.d_xu, &L.d_c2, &L.d_mxu, &L.d_mc2, &L.d_mh2, &L.d_mpart}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    L.nrhs_cap = 0;
    L.mm_groups = 0;
    if (own_stream && L.st) (void)hipStreamDestroy(L.st);
}

static void free_all(hsw_ctx* ctx) {
    drop_graphs(ctx);
    for (size_t l = 0; l < ctx->lanes.size(); ++l) free_lane(ctx->lanes[l], l > 0);
    ctx->lanes.clear();
    for (hipEvent_t& e : ctx->gev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->gst) (void)hipStreamDestroy(ctx->gst);
    void* ptrs[] = {ctx->d_inst, ctx->d_pan, ctx->d_prob, ctx->d_perm, ctx->d_ulist,
                    ctx->d_cmap, ctx->d_pmap, ctx->d_hmap, ctx->d_fwork, ctx->d_sitems, ctx->d_et, ctx->d_c,
                    ctx->d_L, ctx->d_G != ctx->d_L ? ctx->d_G : nullptr, ctx->d_dinv, ctx->d_ws[0],
                    ctx->d_ws[1], ctx->d_err, ctx->d_T};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

// ---------------------------------------------------------------------------
// First column of G the solves read, rounded down to the inversion's 64-column
// blocks.  A leaf front's pivots are ordered plane by plane; on a panel with
// ga auxiliary planes the forward products of its solves start at the first
// pivot of the panel's own planes (the vector is zero before it) and the
// backward pass writes only those pivots (a leaf has no children to feed), so
// the columns of the auxiliary planes are never read and the inversion skips
// their blocks.  Every other front, and every front with full_inverse, is
// formed whole.
static void set_inverse_columns(hsw_ctx* ctx) {
    for (size_t i = 0; i < ctx->inst_h.size(); ++i) {
        FrontInst& f = ctx->inst_h[i];
        f.g0 = 0;
        if (ctx->full_inverse || f.child0 >= 0 || f.child1 >= 0) continue;
        const PanelDev& P = ctx->pan_h[f.panel];
        const int cells = ctx->classes[P.cls].cellw[(int)i - P.inst_base] >> 16;
        f.g0 = std::min(P.ga * cells, f.s) / 64 * 64;
    }
}

// Algorithmic bytes and multiply-adds of the inversion launches and of the
// copies of L_F^{-1}, from the formed columns of every front (s' = s - g0):
// G written for its n rows, the trailing s' x s' part of L_F and the formed
// columns of F_BL read; s'^3/6 + u s'^2/2 complex multiply-adds.
static void inverse_accounting(hsw_ctx* ctx) {
    for (Launch& l : ctx->inv_depth) l.bytes_per_esz = l.cmac = 0;
    for (Launch& l : ctx->lfcopy_depth) l.bytes_per_esz = 0;
    ctx->inv_launch.bytes_per_esz = ctx->inv_launch.cmac = 0;
    ctx->lfcopy_all.bytes_per_esz = 0;
    for (ProbHost& h : ctx->ph) h.inverse_cmac = 0;
    for (const FrontInst& f : ctx->inst_h) {
        const double sd = f.s - f.g0, ud = f.u, nd = f.s + f.u;
        const double bytes = nd * sd + sd * (sd + 1) / 2 + ud * sd;
        const double cmac = sd * sd * sd / 6 + ud * sd * sd / 2;
        ctx->inv_depth[f.depth].bytes_per_esz += bytes;
        ctx->inv_depth[f.depth].cmac += cmac;
        ctx->lfcopy_depth[f.depth].bytes_per_esz += 2.0 * f.s * sd;
        ctx->inv_launch.bytes_per_esz += bytes;
        ctx->inv_launch.cmac += cmac;
        ctx->lfcopy_all.bytes_per_esz += 2.0 * f.s * sd;
        ctx->ph[ctx->pan_h[f.panel].prob].inverse_cmac += cmac;
    }
}

static hsw_status plan_all(hsw_ctx* ctx, const hsw_problem* p, int nprob) {
    std::map<std::tuple<int, int, int>, int> tree_idx;
    std::map<std::tuple<int, int, int, int>, int> cls_idx;
    int64_t c_off = 0;
    for (int k = 0; k < nprob; ++k) {
        const hsw_problem& q = p[k];
        for (int j = 0; j < 3; ++j)
            if (q.n[j] < 1) return fail(ctx, HSW_E_INVAL, "n must be positive");
        if (!(q.h > 0) || !(q.omega > 0) || !(q.alpha >= 0) || !(q.pml_amp >= 0) ||
            !std::isfinite(q.h) || !std::isfinite(q.omega) || !std::isfinite(q.alpha) ||
            !std::isfinite(q.pml_amp))
            return fail(ctx, HSW_E_INVAL, "h, omega must be positive; alpha, pml_amp >= 0");
        if (q.gamma < 1 || q.panel_depth < 1 || q.leaf < 2)
            return fail(ctx, HSW_E_INVAL, "gamma >= 1, panel_depth >= 1, leaf >= 2 required");
        ProbHost h;
        for (int j = 0; j < 3; ++j) h.N[j] = q.n[j] + 2 * q.gamma;
        h.Npad = (int64_t)h.N[0] * h.N[1] * h.N[2];
        h.Nint = (int64_t)q.n[0] * q.n[1] * q.n[2];
        if (h.Npad > (int64_t)1 << 31) return fail(ctx, HSW_E_INVAL, "grid too large");
        h.m = (q.n[2] + q.panel_depth - 1) / q.panel_depth;
        h.panel_base = (int)ctx->pan_h.size();
        h.c_off = c_off;
        c_off += h.Nint;
        auto tk = std::make_tuple(h.N[0], h.N[1], q.leaf);
        if (!tree_idx.count(tk)) {
            tree_idx[tk] = (int)ctx->trees.size();
            ctx->trees.push_back(build_lateral_tree(h.N[0], h.N[1], q.leaf));
        }
        const int ti = tree_idx[tk];
        for (int i = 0; i < h.m; ++i) {
            PanelDev P{};
            P.prob = k;
            P.Nx = h.N[0];
            P.Ny = h.N[1];
            P.lo = i == 0 ? 0 : q.gamma + i * q.panel_depth;
            P.hi = i == h.m - 1 ? h.N[2] : q.gamma + (i + 1) * q.panel_depth;
            P.ga = i == 0 ? 0 : q.gamma;
            P.nz = P.ga + P.hi - P.lo;
            auto ck = std::make_tuple(h.N[0], h.N[1], P.nz, q.leaf);
            if (!cls_idx.count(ck)) {
                PanelClass pc;
                std::string e = build_class(ctx->trees[ti], P.nz, pc);
                if (!e.empty()) return fail(ctx, HSW_E_INVAL, "plan: " + e);
                cls_idx[ck] = (int)ctx->classes.size();
                ctx->classes.push_back(std::move(pc));
            }
            P.cls = cls_idx[ck];
            ctx->pan_h.push_back(P);
        }
        ctx->ph.push_back(h);
    }
    // class arrays, concatenated
    int po = 0, uo = 0, mo = 0, pmo = 0;
    for (auto& c : ctx->classes) {
        ctx->cls_perm_off.push_back(po);
        ctx->cls_ulist_off.push_back(uo);
        ctx->cls_cmap_off.push_back(mo);
        ctx->cls_pmap_off.push_back(pmo);
        po += c.naux;
        uo += (int)c.ulist.size();
        mo += (int)c.cmap.size();
        pmo += (int)c.pmap.size();
        ctx->max_naux = std::max(ctx->max_naux, c.naux);
        ctx->max_wsize = std::max(ctx->max_wsize, c.wsize);
        ctx->max_c2 = std::max(ctx->max_c2, c.c2size);
        ctx->cls_c2_base.push_back(ctx->total_c2);
        ctx->total_c2 += c.c2size;
        ctx->total_naux += c.naux;
        ctx->maxdepth = std::max(ctx->maxdepth, c.maxdepth);
    }
    // front instances
    int64_t loff = 0, doff = 0;
    for (size_t g = 0; g < ctx->pan_h.size(); ++g) {
        PanelDev& P = ctx->pan_h[g];
        const PanelClass& c = ctx->classes[P.cls];
        P.perm_off = ctx->cls_perm_off[P.cls];
        P.inst_base = (int)ctx->inst_h.size();
        P.nfront = c.nfront;
        ProbHost& h = ctx->ph[P.prob];
        h.setup_cmac += c.factor_cmac;
        h.factor_entries += c.lsize;
        h.levels = std::max(h.levels, c.maxdepth + 1);
        for (int f = 0; f < c.nfront; ++f) {
            FrontInst fi{};
            fi.s = c.s[f];
            fi.u = c.u[f];
            fi.start = c.start[f];
            fi.wvoff = c.woff[f];
            fi.child0 = c.child0[f] >= 0 ? P.inst_base + c.child0[f] : -1;
            fi.child1 = c.child1[f] >= 0 ? P.inst_base + c.child1[f] : -1;
            fi.cw0 = c.child0[f] >= 0 ? c.woff[c.child0[f]] : 0;
            fi.cw1 = c.child1[f] >= 0 ? c.woff[c.child1[f]] : 0;
            fi.uoff = ctx->cls_ulist_off[P.cls] + c.uoff[f];
            fi.moff = ctx->cls_cmap_off[P.cls] + c.moff[f];
            fi.panel = (int)g;
            fi.depth = c.depth[f];
            fi.loff = loff;
            fi.doff = doff;
            loff += (int64_t)(fi.s + fi.u) * fi.s;
            doff += fi.s;
            ctx->inst_h.push_back(fi);
        }
    }
    set_inverse_columns(ctx);
    ctx->L_size = loff;
    ctx->D_size = doff;
    return HSW_OK;
}

// Workgroups of a launch go to the chip's XCDs round-robin (workgroup b to
// XCD b mod 8), each XCD with its own L2.  Reorder the items [b, e) of a
// launch so that the items of one front land on one XCD, consecutively, and
// share the front's data in that L2: fronts go to the least loaded of eight
// bins, and slot p takes the next item of bin p mod 8 (or, once that bin is
// empty, of the fullest bin).
template <typename W, typename K>
static void xcd_group_by(std::vector<W>& w, size_t b, size_t e, K key) {
    constexpr int X = 8;
    if (e - b <= 1) return;
    std::map<int64_t, std::vector<W>> by;
    std::vector<int64_t> order;
    for (size_t i = b; i < e; ++i) {
        const int64_t k = key(w[i]);
        if (!by.count(k)) order.push_back(k);
        by[k].push_back(w[i]);
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t c) { return by[a].size() > by[c].size(); });
    std::vector<std::vector<W>> bins(X);
    for (int64_t f : order) {
        int x = 0;
        for (int y = 1; y < X; ++y)
            if (bins[y].size() < bins[x].size()) x = y;
        bins[x].insert(bins[x].end(), by[f].begin(), by[f].end());
    }
    std::vector<size_t> pos(X, 0);
    for (size_t p = b; p < e; ++p) {
        int x = (int)((p - b) % X);
        if (pos[x] == bins[x].size()) {
            x = 0;
            for (int y = 1; y < X; ++y)
                if (bins[y].size() - pos[y] > bins[x].size() - pos[x]) x = y;
        }
        w[p] = bins[x][pos[x]++];
    }
}

static void xcd_group(std::vector<int2>& w, size_t b, size_t e) {
    xcd_group_by(w, b, e, [](const int2& v) { return (int64_t)v.x; });
}

static void schedule_all(hsw_ctx* ctx, std::vector<int2>& fwork, std::vector<SolveItem>& sitems);

// Complex multiply-adds of one sweep application per right-hand side (Alg.
// 1.5: 2m - 1 panel solves), from the G entries the passes need: panel i's
// solve of the forward sweep reads leaves from the panel's own planes in both
// passes; its coupling solve of the backward sweep (i < m - 1) reads them from
// the last plane in the forward pass.
static void apply_accounting(hsw_ctx* ctx) {
    for (ProbHost& h : ctx->ph) {
        h.apply_cmac = 0;
        for (int i = 0; i < h.m; ++i) {
            const PanelDev& P = ctx->pan_h[h.panel_base + i];
            for (const SolveLevel& l : ctx->slevels[P.cls]) {
                h.apply_cmac += 2 * l.g_need(P.ga);
                if (i < h.m - 1) h.apply_cmac += l.g_need(P.nz - 1) + l.g_need(P.ga);
            }
        }
    }
}

static void schedule_all(hsw_ctx* ctx, std::vector<int2>& fwork, std::vector<SolveItem>& sitems) {
    const int D = ctx->maxdepth;
    std::vector<std::vector<int>> at(D + 1);
    for (size_t i = 0; i < ctx->inst_h.size(); ++i) at[ctx->inst_h[i].depth].push_back((int)i);
    ctx->fsched.assign(D + 1, DepthSchedule{});
    for (int d = D; d >= 0; --d) {
        DepthSchedule& ds = ctx->fsched[d];
        int64_t woff = 0;
        int smax = 0;
        for (int i : at[d]) {
            FrontInst& f = ctx->inst_h[i];
            f.woff = woff;
            woff += (int64_t)f.u * f.u;
            smax = std::max(smax, f.s);
        }
        ctx->ws_size[d & 1] = std::max(ctx->ws_size[d & 1], woff);
        ds.assemble.off = (int64_t)fwork.size();
        for (int i : at[d]) {
            const FrontInst& f = ctx->inst_h[i];
            int nt = (f.s + f.u + TILE - 1) / TILE;
            for (int t = 0; t < nt * (nt + 1) / 2; ++t) fwork.push_back(make_int2(i, t));
        }
        ds.assemble.count = (int)(fwork.size() - ds.assemble.off);
        xcd_group(fwork, ds.assemble.off, fwork.size());
        for (int i : at[d]) {
            const FrontInst& f = ctx->inst_h[i];
            const double n = f.s + f.u;
            ds.assemble.bytes_per_esz += n * (n + 1) / 2;  // the front is written once
            for (int c : {f.child0, f.child1})
                if (c >= 0) {
                    const double uc = ctx->inst_h[c].u;
                    ds.assemble.bytes_per_esz += uc * (uc + 1) / 2;  // child update pulled
                }
        }
        for (int k = 0; k < smax; k += NB) {
            Launch l{(int64_t)fwork.size(), 0, k};
            for (int i : at[d])
                if (ctx->inst_h[i].s > k) fwork.push_back(make_int2(i, 0));
            l.count = (int)(fwork.size() - l.off);
            for (int i : at[d]) {
                const FrontInst& f = ctx->inst_h[i];
                if (f.s <= k) continue;
                const double b = std::min(NB, f.s - k);
                l.bytes_per_esz += b * (b + 1) + b;  // block read + written, reciprocal pivots
                l.cmac += b * b * b / 6;
            }
            ds.ldlt.push_back(l);
            Launch pl{(int64_t)fwork.size(), 0, k};
            for (int i : at[d]) {
                const FrontInst& f = ctx->inst_h[i];
                if (f.s <= k) continue;
                int b = std::min(NB, f.s - k);
                int nrb = (f.s + f.u - k - b + 63) / 64;
                for (int rb = 0; rb < nrb; ++rb) fwork.push_back(make_int2(i, rb));
            }
            pl.count = (int)(fwork.size() - pl.off);
            xcd_group(fwork, pl.off, fwork.size());
            for (int i : at[d]) {
                const FrontInst& f = ctx->inst_h[i];
                if (f.s <= k) continue;
                const double b = std::min(NB, f.s - k);
                const double rows = f.s + f.u - k - b;
                pl.bytes_per_esz += 2 * rows * b + b * b / 2 + b;
                pl.cmac += rows * b * b / 2;
            }
            ds.panel.push_back(pl);
            Launch t{(int64_t)fwork.size(), 0, k};
            for (int i : at[d]) {
                const FrontInst& f = ctx->inst_h[i];
                if (f.s <= k) continue;
                int b = std::min(NB, f.s - k);
                int tr = f.s + f.u - k - b;
                if (tr <= 0) continue;
                int nt = (tr + TILE - 1) / TILE;
                for (int q = 0; q < nt * (nt + 1) / 2; ++q) fwork.push_back(make_int2(i, q));
            }
            t.count = (int)(fwork.size() - t.off);
            xcd_group(fwork, t.off, fwork.size());
            for (int i : at[d]) {
                const FrontInst& f = ctx->inst_h[i];
                if (f.s <= k) continue;
                const double b = std::min(NB, f.s - k);
                const double tr = f.s + f.u - k - b;
                if (tr <= 0) continue;
                t.bytes_per_esz += tr * (tr + 1) + tr * b;  // lower triangle read+written, panel read
                t.cmac += tr * (tr + 1) / 2 * b;
            }
            ds.trail.push_back(t);
            Launch pv{(int64_t)fwork.size(), 0, k};
            for (int i : at[d]) {
                const FrontInst& f = ctx->inst_h[i];
                if (f.s <= k) continue;
                const int b = std::min(NB, f.s - k);
                const int tr = f.s + f.u - k - b, tc = f.s - k - b;
                if (tr <= 0 || tc <= 0) continue;
                const int nt = (tr + TILE - 1) / TILE, ntc = (tc + TILE - 1) / TILE;
                for (int q = 0; q < nt * (nt + 1) / 2; ++q) {
                    int ti, tj;
                    tri_decode(q, ti, tj);
                    if (tj < ntc) fwork.push_back(make_int2(i, q));
                }
                const double bd = b, trd = tr, tcd = tc;
                const double ent = tcd * (tcd + 1) / 2 + (trd - tcd) * tcd;  // lower part of the pivot columns
                pv.bytes_per_esz += 2 * ent + trd * bd + tcd * bd;
                pv.cmac += ent * bd;
            }
            pv.count = (int)(fwork.size() - pv.off);
            xcd_group(fwork, pv.off, fwork.size());
            ds.pivots.push_back(pv);
            Launch lf{(int64_t)fwork.size(), 0, k};
            if (k > 0) {
                for (int i : at[d]) {
                    const FrontInst& f = ctx->inst_h[i];
                    if (f.s <= k) continue;
                    const int nrt = (f.s + f.u - k + TILE - 1) / TILE;
                    for (int q = 0; q < nrt; ++q) fwork.push_back(make_int2(i, q));
                    const double b = std::min(NB, f.s - k), rows = f.s + f.u - k;
                    lf.bytes_per_esz += 2 * (rows * b - b * (b - 1) / 2) + (rows + b) * k;
                    lf.cmac += (rows * b - b * (b - 1) / 2) * k;
                }
            }
            lf.count = (int)(fwork.size() - lf.off);
            xcd_group(fwork, lf.off, fwork.size());
            ds.left.push_back(lf);
        }
        ds.schur = Launch{(int64_t)fwork.size(), 0, 0};
        for (int i : at[d]) {
            const FrontInst& f = ctx->inst_h[i];
            if (f.u <= 0) continue;
            const int nt = (f.u + TILE - 1) / TILE;
            for (int q = 0; q < nt * (nt + 1) / 2; ++q) fwork.push_back(make_int2(i, q));
            const double sd = f.s, ud = f.u;
            ds.schur.bytes_per_esz += ud * (ud + 1) + ud * sd;  // F_BR lower read + written, F_BL read
            ds.schur.cmac += ud * (ud + 1) / 2 * sd;
        }
        ds.schur.count = (int)(fwork.size() - ds.schur.off);
        xcd_group(fwork, ds.schur.off, fwork.size());
        ds.nfronts = (int)at[d].size();
    }
    // selective inversion, one launch per depth (the fronts of a depth over all
    // panels and problems), each followed by the copy of L_F^{-1} from the
    // depth's scratch over L_F when the inverse overwrites the factor
    ctx->inv_depth.assign(D + 1, Launch{0, 0, 0});
    ctx->lfcopy_depth.assign(D + 1, Launch{0, 0, 0});
    ctx->inv_launch = Launch{0, 0, 0};
    ctx->inv_scratch = 0;
    for (int d = D; d >= 0; --d) {
        Launch& il = ctx->inv_depth[d];
        il.off = (int64_t)fwork.size();
        int64_t toff = 0;
        for (int i : at[d]) {
            FrontInst& f = ctx->inst_h[i];
            f.toff = toff;
            toff += (int64_t)f.s * f.s;
            const int nrb = (f.s + f.u + 63) / 64;
            for (int rb = 0; rb < nrb; ++rb) fwork.push_back(make_int2(i, rb));
        }
        il.count = (int)(fwork.size() - il.off);
        xcd_group(fwork, il.off, fwork.size());
        ctx->inv_scratch = std::max(ctx->inv_scratch, toff);
        Launch& cl = ctx->lfcopy_depth[d];
        cl.off = (int64_t)fwork.size();
        for (int i : at[d]) {
            const FrontInst& f = ctx->inst_h[i];
            for (int rb = 0; rb < (f.s + 63) / 64; ++rb) fwork.push_back(make_int2(i, rb));
        }
        cl.count = (int)(fwork.size() - cl.off);
    }
    // the one-launch layout: every front, long rows first in the XCD order
    ctx->toff_all.assign(ctx->inst_h.size(), 0);
    ctx->inv_scratch_all = 0;
    ctx->inv_launch.off = (int64_t)fwork.size();
    for (size_t i = 0; i < ctx->inst_h.size(); ++i) {
        const FrontInst& f = ctx->inst_h[i];
        ctx->toff_all[i] = ctx->inv_scratch_all;
        ctx->inv_scratch_all += (int64_t)f.s * f.s;
        for (int rb = 0; rb < (f.s + f.u + 63) / 64; ++rb) fwork.push_back(make_int2((int)i, rb));
    }
    ctx->inv_launch.count = (int)(fwork.size() - ctx->inv_launch.off);
    xcd_group(fwork, ctx->inv_launch.off, fwork.size());
    ctx->lfcopy_all.off = (int64_t)fwork.size();
    for (size_t i = 0; i < ctx->inst_h.size(); ++i)
        for (int rb = 0; rb < (ctx->inst_h[i].s + 63) / 64; ++rb) fwork.push_back(make_int2((int)i, rb));
    ctx->lfcopy_all.count = (int)(fwork.size() - ctx->lfcopy_all.off);
    // solve work lists per class and depth
    ctx->slevels.assign(ctx->classes.size(), {});
    for (size_t ci = 0; ci < ctx->classes.size(); ++ci) {
        const PanelClass& c = ctx->classes[ci];
        ctx->slevels[ci].assign(c.maxdepth + 1, SolveLevel{});
        for (int d = 0; d <= c.maxdepth; ++d) {
            SolveLevel& sl = ctx->slevels[ci][d];
            auto item = [&](int f, int blk) {
                SolveItem it{};
                it.loff = c.loff[f];
                it.n = c.s[f] + c.u[f];
                it.s = c.s[f];
                it.start = c.start[f];
                it.blk = blk;
                it.moff = ctx->cls_cmap_off[ci] + c.moff[f];
                it.c2 = c.c2off[f];
                const int p = c.parent[f];
                it.push = p < 0 ? -1 : c.c2off[p] + (c.child0[p] == f ? 0 : c.s[p] + c.u[p]);
                it.pmap = ctx->cls_pmap_off[ci] + c.pmoff[f];
                it.xu = c.woff[f];
                it.cxu0 = c.child0[f] >= 0 ? c.woff[c.child0[f]] : -1;
                it.cxu1 = c.child1[f] >= 0 ? c.woff[c.child1[f]] : -1;
                it.cell0 = c.cell0[f];
                it.cellw = c.cellw[f];
                it.leaf = c.child0[f] < 0 && c.child1[f] < 0;
                return it;
            };
            for (int k = 0; k < N_FWD_SHAPES; ++k) {
                const int rb = FWD_SHAPES[k].block;
                sl.foff[k] = (int64_t)sitems.size();
                for (int f : c.at_depth[d])
                    for (int blk = 0; blk < c.s[f] + c.u[f]; blk += rb) sitems.push_back(item(f, blk));
                sl.fcount[k] = (int)(sitems.size() - sl.foff[k]);
                // the row blocks of one front on one XCD: their shared cache
                // lines and the staged front vector hit that XCD's L2
                xcd_group_by(sitems, sl.foff[k], sitems.size(), [](const SolveItem& q) { return q.loff; });
            }
            sl.toff = (int64_t)sitems.size();
            for (int f : c.at_depth[d]) sitems.push_back(item(f, 0));
            sl.tcount = (int)(sitems.size() - sl.toff);
            xcd_group_by(sitems, sl.toff, sitems.size(), [](const SolveItem& q) { return q.loff; });
            for (int k = 0; k < N_BWD_SHAPES; ++k) {
                const int cb = BWD_SHAPES[k].block;
                sl.boff[k] = (int64_t)sitems.size();
                for (int f : c.at_depth[d])
                    for (int blk = 0; blk < c.s[f]; blk += cb) sitems.push_back(item(f, blk));
                sl.bcount[k] = (int)(sitems.size() - sl.boff[k]);
                xcd_group_by(sitems, sl.boff[k], sitems.size(), [](const SolveItem& q) { return q.loff; });
            }
            sl.g_leaf.assign(c.nz + 1, 0.0);
            sl.fwd_vec.assign(c.nz + 1, 0.0);
            sl.bwd_vec.assign(c.nz + 1, 0.0);
            const double es = ctx->esz;
            for (int f : c.at_depth[d]) {
                const bool leaf = c.child0[f] < 0 && c.child1[f] < 0;
                const int cells = c.cellw[f] >> 16;  // pivots per plane (pivots are plane-major)
                if (leaf) {
                    for (int p = 0; p <= c.nz; ++p) {
                        const double r = std::max(0, c.s[f] - p * cells);
                        sl.g_leaf[p] += r * (r + 1) / 2 + (double)c.u[f] * r;
                    }
                } else {
                    sl.g_inner += (double)c.s[f] * (c.s[f] + 1) / 2 + (double)c.u[f] * c.s[f];
                }
                sl.smax = std::max(sl.smax, c.s[f]);
                sl.nmax = std::max(sl.nmax, c.s[f] + c.u[f]);
                double uc = 0;
                for (int ch : {c.child0[f], c.child1[f]})
                    if (ch >= 0) uc += c.u[ch];
                for (int p = 0; p <= c.nz; ++p) {
                    // pivots on the panel's own planes (p auxiliary planes
                    // below them), and the pivots the forward pass carries: a
                    // leaf's auxiliary pivots have zero right-hand sides and
                    // no children, so they stay zero
                    const double grid = std::max(0, c.s[f] - p * cells);
                    const double live = leaf ? grid : c.s[f];
                    // forward: v_S read (right-hand side with the children's
                    // parts added), the children's contributions, x_S and the
                    // update part written
                    sl.fwd_vec[p] += es * (2 * live + uc + c.u[f]);
                    // backward: [x_S; -x_U] read, the children's update-set
                    // values written, x_S to the grid (complex128)
                    sl.bwd_vec[p] += es * (live + c.u[f] + uc) + 16 * grid;
                }
            }
            const int dflt = sl.nmax >= SOLVE_SMALL_BLOCK_N ? 1 : 0;
            for (int key = 0; key < N_RHS_KEYS; ++key) sl.fsel[key] = sl.bsel[key] = dflt;
        }
    }
}

// ---------------------------------------------------------------------------
extern "C" hsw_status hsw_create(const hsw_problem* p, int32_t nprob, hsw_precision prec,
                                 void* stream, hsw_ctx** out) {
    if (!out) return HSW_E_INVAL;
    *out = nullptr;
    if (!p || nprob < 1) {
        g_create_error = "need at least one problem";
        return HSW_E_INVAL;
    }
    if (prec != HSW_C128 && prec != HSW_C64 && prec != HSW_C64_BF16GEMM) {
        g_create_error = "unknown precision";
        return HSW_E_INVAL;
    }
    hsw_ctx* ctx = new hsw_ctx();
    ctx->st = (hipStream_t)stream;
    ctx->lanes.resize(1);
    ctx->lanes[0].st = ctx->st;
    if (hipGetDevice(&ctx->device) != hipSuccess) ctx->device = 0;
    if (const char* at = std::getenv("HSW_AUTOTUNE")) ctx->autotune = std::string(at) != "0";
    if (const char* tr = std::getenv("HSW_TUNE_REPORT")) ctx->tune_report = std::string(tr) != "0";
    ctx->prec = prec;
    ctx->esz = prec == HSW_C128 ? 16 : 8;
    ctx->probs.assign(p, p + nprob);
    for (hsw_problem& q : ctx->probs)
        if (q.leaf == 0) q.leaf = DEFAULT_LEAF;
    hsw_status s = plan_all(ctx, ctx->probs.data(), nprob);
    if (s != HSW_OK) {
        g_create_error = ctx->err;
        delete ctx;
        return s;
    }
    std::vector<int2> fwork;
    std::vector<SolveItem> sitems;
    schedule_all(ctx, fwork, sitems);
    inverse_accounting(ctx);
    apply_accounting(ctx);
    // stretch tables: per problem 3 axes, per panel one x3 table
    int64_t eo = 0;
    for (size_t k = 0; k < ctx->ph.size(); ++k) {
        ctx->et_prob_off.push_back(eo);
        for (int j = 0; j < 3; ++j) eo += 2 * ctx->ph[k].N[j] + 1;
    }
    for (auto& P : ctx->pan_h) {
        P.e3_off = (int32_t)eo;
        ctx->et_panel_off.push_back(eo);
        eo += 2 * P.nz + 1;
    }
    ctx->et_size = eo;
    for (size_t k = 0; k < ctx->ph.size(); ++k) {
        ProbDev Q{};
        const hsw_problem& q = ctx->probs[k];
        for (int j = 0; j < 3; ++j) {
            Q.n[j] = q.n[j];
            Q.N[j] = ctx->ph[k].N[j];
        }
        Q.gamma = q.gamma;
        Q.Npad = ctx->ph[k].Npad;
        Q.h = q.h;
        Q.omega = q.omega;
        Q.alpha = q.alpha;
        int64_t o = ctx->et_prob_off[k];
        for (int j = 0; j < 3; ++j) {
            Q.e_off[j] = (int32_t)o;
            o += 2 * Q.N[j] + 1;
        }
        Q.c = nullptr;  // set after allocation
        ctx->prob_h.push_back(Q);
    }
    // memory sizing, checked before any allocation
    int64_t nint_total = 0;
    for (auto& h : ctx->ph) nint_total += h.Nint;
    size_t ints = 0;
    for (auto& c : ctx->classes)
        ints += (size_t)c.naux + c.ulist.size() + c.cmap.size() + c.pmap.size();
    // the factor block holds L during the factorisation and G after the
    // in-place selective inversion; the scratch holds L_F^{-1} of every front
    // (one inversion launch) or, when that does not fit, of one depth
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) {
        g_create_error = "hipMemGetInfo failed (no device?)";
        delete ctx;
        return HSW_E_DEVICE;
    }
    // the fastest layout that fits: a separate G block (no scratch, no copy),
    // else in place with every L_F^{-1} in the scratch, else in place one
    // depth at a time
    const size_t base = (size_t)ctx->esz * (ctx->L_size + ctx->D_size + ctx->ws_size[0] + ctx->ws_size[1]);
    const size_t room = freeb / 100 * 90;
    ctx->keep_factors = base + (size_t)ctx->esz * ctx->L_size <= room;
    ctx->inv_by_depth = !ctx->keep_factors && base + (size_t)ctx->esz * ctx->inv_scratch_all > room;
    if (!ctx->inv_by_depth) {
        for (size_t i = 0; i < ctx->inst_h.size(); ++i) ctx->inst_h[i].toff = ctx->toff_all[i];
        ctx->inv_scratch = ctx->inv_scratch_all;
    }
    const size_t need = base + (size_t)ctx->esz * (ctx->keep_factors ? ctx->L_size : ctx->inv_scratch) +
                        sizeof(FrontInst) * ctx->inst_h.size() + sizeof(PanelDev) * ctx->pan_h.size() +
                        sizeof(ProbDev) * ctx->prob_h.size() + 4 * ints + 8 * fwork.size() +
                        sizeof(SolveItem) * sitems.size() + 16 * (size_t)eo + 8 * (size_t)nint_total;
    if (need > freeb / 100 * 95) {
        char buf[256];
        snprintf(buf, sizeof buf, "plan needs %.3f GB of device memory, %.3f GB free",
                 need / 1e9, freeb / 1e9);
        g_create_error = buf;
        delete ctx;
        return HSW_E_NOMEM;
    }
#define ACHK(expr)                                                      \
    do {                                                                \
        hipError_t e_ = (expr);                                         \
        if (e_ != hipSuccess) {                                         \
            g_create_error = std::string(#expr) + ": " + hipGetErrorString(e_); \
            free_all(ctx);                                              \
            delete ctx;                                                 \
            return HSW_E_DEVICE;                                        \
        }                                                               \
    } while (0)
    ACHK(dalloc(&ctx->d_c, 8 * (size_t)nint_total));
    for (size_t k = 0; k < ctx->prob_h.size(); ++k) ctx->prob_h[k].c = ctx->d_c + ctx->ph[k].c_off;
    ACHK(dalloc(&ctx->d_inst, sizeof(FrontInst) * ctx->inst_h.size()));
    ACHK(dalloc(&ctx->d_pan, sizeof(PanelDev) * ctx->pan_h.size()));
    ACHK(dalloc(&ctx->d_prob, sizeof(ProbDev) * ctx->prob_h.size()));
    std::vector<int> perm, ul, cm, pm, hm;
    for (auto& c : ctx->classes) {
        perm.insert(perm.end(), c.perm.begin(), c.perm.end());
        ul.insert(ul.end(), c.ulist.begin(), c.ulist.end());
        cm.insert(cm.end(), c.cmap.begin(), c.cmap.end());
        pm.insert(pm.end(), c.pmap.begin(), c.pmap.end());
        hm.insert(hm.end(), c.hmap.begin(), c.hmap.end());
    }
    ACHK(dalloc(&ctx->d_perm, 4 * perm.size()));
    ACHK(dalloc(&ctx->d_ulist, 4 * std::max<size_t>(ul.size(), 1)));
    ACHK(dalloc(&ctx->d_cmap, 4 * std::max<size_t>(cm.size(), 1)));
    ACHK(dalloc(&ctx->d_fwork, 8 * std::max<size_t>(fwork.size(), 1)));
    ACHK(dalloc(&ctx->d_pmap, 4 * std::max<size_t>(pm.size(), 1)));
    ACHK(dalloc(&ctx->d_hmap, 4 * std::max<size_t>(hm.size(), 1)));
    ACHK(dalloc(&ctx->d_sitems, sizeof(SolveItem) * std::max<size_t>(sitems.size(), 1)));
    ACHK(dalloc(&ctx->d_et, 16 * (size_t)eo));
    ACHK(dalloc(&ctx->d_L, (size_t)ctx->esz * ctx->L_size));
    if (ctx->keep_factors) {
        ACHK(dalloc(&ctx->d_G, (size_t)ctx->esz * ctx->L_size));
    } else {
        ctx->d_G = ctx->d_L;
        ACHK(dalloc(&ctx->d_T, (size_t)ctx->esz * std::max<int64_t>(ctx->inv_scratch, 1)));
    }
    ACHK(dalloc(&ctx->d_dinv, (size_t)ctx->esz * ctx->D_size));
    ACHK(dalloc(&ctx->d_ws[0], (size_t)ctx->esz * std::max<int64_t>(ctx->ws_size[0], 1)));
    ACHK(dalloc(&ctx->d_ws[1], (size_t)ctx->esz * std::max<int64_t>(ctx->ws_size[1], 1)));
    ACHK(dalloc(&ctx->d_err, 2 * sizeof(int)));
    hipStream_t st = ctx->st;
    ACHK(hipMemcpyAsync(ctx->d_inst, ctx->inst_h.data(), sizeof(FrontInst) * ctx->inst_h.size(),
                        hipMemcpyHostToDevice, st));
    ACHK(hipMemcpyAsync(ctx->d_pan, ctx->pan_h.data(), sizeof(PanelDev) * ctx->pan_h.size(),
                        hipMemcpyHostToDevice, st));
    ACHK(hipMemcpyAsync(ctx->d_prob, ctx->prob_h.data(), sizeof(ProbDev) * ctx->prob_h.size(),
                        hipMemcpyHostToDevice, st));
    ACHK(hipMemcpyAsync(ctx->d_perm, perm.data(), 4 * perm.size(), hipMemcpyHostToDevice, st));
    if (!ul.empty())
        ACHK(hipMemcpyAsync(ctx->d_ulist, ul.data(), 4 * ul.size(), hipMemcpyHostToDevice, st));
    if (!cm.empty())
        ACHK(hipMemcpyAsync(ctx->d_cmap, cm.data(), 4 * cm.size(), hipMemcpyHostToDevice, st));
    if (!fwork.empty())
        ACHK(hipMemcpyAsync(ctx->d_fwork, fwork.data(), 8 * fwork.size(), hipMemcpyHostToDevice, st));
    if (!pm.empty())
        ACHK(hipMemcpyAsync(ctx->d_pmap, pm.data(), 4 * pm.size(), hipMemcpyHostToDevice, st));
    if (!hm.empty())
        ACHK(hipMemcpyAsync(ctx->d_hmap, hm.data(), 4 * hm.size(), hipMemcpyHostToDevice, st));
    if (!sitems.empty())
        ACHK(hipMemcpyAsync(ctx->d_sitems, sitems.data(), sizeof(SolveItem) * sitems.size(),
                            hipMemcpyHostToDevice, st));
    ACHK(hipStreamSynchronize(st));
#undef ACHK
    *out = ctx;
    return HSW_OK;
}

extern "C" void hsw_destroy(hsw_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->st);
    free_all(ctx);
    delete ctx;
}

extern "C" hsw_status hsw_set_option(hsw_ctx* ctx, const char* key, int64_t value) {
    if (!ctx || !key) return HSW_E_INVAL;
    const std::string k(key);
    if (k == "graph") {
        ctx->use_graph = value != 0;
    } else if (k == "autotune") {
        ctx->autotune = value != 0;
    } else if (k == "solve_lanes") {
        if (value < 1 || value > 16) return fail(ctx, HSW_E_INVAL, "solve_lanes is 1..16");
        ctx->nlanes = (int)value;
    } else if (k == "block_gmres") {
        ctx->block_gmres = value != 0;
    } else if (k == "gmres_device_test") {
        ctx->gmres_device_test = value != 0;
    } else if (k == "bf16_mfma") {
        ctx->bf16_mfma = value != 0;
        ctx->factored = false;
    } else if (k == "inverse_by_depth") {
        const bool by = value != 0;
        if (by != ctx->inv_by_depth) {
            int64_t need = 0;
            std::vector<FrontInst> inst = ctx->inst_h;
            if (by) {
                std::vector<int64_t> off(ctx->maxdepth + 1, 0);
                for (auto& f : inst) {
                    f.toff = off[f.depth];
                    off[f.depth] += (int64_t)f.s * f.s;
                }
                for (int64_t o : off) need = std::max(need, o);
            } else {
                for (size_t i = 0; i < inst.size(); ++i) inst[i].toff = ctx->toff_all[i];
                need = ctx->inv_scratch_all;
            }
            if (need > ctx->inv_scratch) {
                void* t = nullptr;
                if (hipMalloc(&t, (size_t)ctx->esz * need) != hipSuccess) {
                    (void)hipGetLastError();
                    return fail(ctx, HSW_E_NOMEM, "inverse_by_depth: no room for the scratch");
                }
                HIPCHK(hipStreamSynchronize(ctx->st));
                (void)hipFree(ctx->d_T);
                ctx->d_T = t;
                ctx->inv_scratch = need;
            }
            HIPCHK(hipMemcpyAsync(ctx->d_inst, inst.data(), sizeof(FrontInst) * inst.size(),
                                  hipMemcpyHostToDevice, ctx->st));
            HIPCHK(hipStreamSynchronize(ctx->st));
            ctx->inst_h = inst;
            ctx->inv_by_depth = by;
            ctx->factored = false;
        }
    } else if (k == "triangular_solves") {
        if (value < 0 || value > 2) return fail(ctx, HSW_E_INVAL, "triangular_solves is 0, 1 or 2");
        ctx->tri_mode = (int)value;
        for (bool& t : ctx->tuned) t = false;
    } else if (k == "full_inverse") {
        const bool full = value != 0;
        if (full != ctx->full_inverse) {
            ctx->full_inverse = full;
            set_inverse_columns(ctx);
            inverse_accounting(ctx);
            HIPCHK(hipMemcpyAsync(ctx->d_inst, ctx->inst_h.data(), sizeof(FrontInst) * ctx->inst_h.size(),
                                  hipMemcpyHostToDevice, ctx->st));
            HIPCHK(hipStreamSynchronize(ctx->st));
            ctx->factored = false;
        }
    } else if (k == "keep_factors") {
        const bool keep = value != 0;
        if (keep != ctx->keep_factors) {
            if (keep) {
                void* g = nullptr;
                if (hipMalloc(&g, (size_t)ctx->esz * std::max<int64_t>(ctx->L_size, 1)) != hipSuccess) {
                    (void)hipGetLastError();
                    return fail(ctx, HSW_E_NOMEM, "keep_factors: no room for a separate G block");
                }
                ctx->d_G = g;
            } else {
                if (!ctx->d_T) {
                    void* t = nullptr;
                    if (hipMalloc(&t, (size_t)ctx->esz * std::max<int64_t>(ctx->inv_scratch, 1)) != hipSuccess) {
                        (void)hipGetLastError();
                        return fail(ctx, HSW_E_NOMEM, "keep_factors 0: no room for the scratch");
                    }
                    ctx->d_T = t;
                }
                HIPCHK(hipStreamSynchronize(ctx->st));
                (void)hipFree(ctx->d_G);
                ctx->d_G = ctx->d_L;
            }
            ctx->keep_factors = keep;
            ctx->factored = false;  // G is rebuilt by the next setup
            for (bool& t : ctx->tuned) t = false;  // the triangular passes come and go with the factors
            drop_graphs(ctx);
        }
    } else if (k == "mm_min_rhs") {
        if (value < 1 || value > MM_MIN_RHS) return fail(ctx, HSW_E_INVAL, "mm_min_rhs is 1..16");
        ctx->mm_min_rhs = (int)value;
    } else if (k == "mm_fwd_form") {
        if (value < -1 || value > 7) return fail(ctx, HSW_E_INVAL, "mm_fwd_form is -1..7");
        ctx->mm_fwd_form = (int)value;
    } else if (k == "mm_bwd_form") {
        if (value < -1 || value > 8) return fail(ctx, HSW_E_INVAL, "mm_bwd_form is -1..8");
        ctx->mm_bwd_form = (int)value;
    } else if (k == "update_order") {
        if (value < -1 || value > 2) return fail(ctx, HSW_E_INVAL, "update_order is -1, 0, 1 or 2");
        ctx->update_order = (int)value;
    } else {
        return fail(ctx, HSW_E_INVAL, "unknown option " + k);
    }
    return HSW_OK;
}

extern "C" const char* hsw_last_error(const hsw_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

extern "C" hsw_status hsw_assemble(hsw_ctx* ctx, const double* const* c) {
    if (!ctx) return HSW_E_INVAL;
    if (!c) return fail(ctx, HSW_E_INVAL, "c is NULL");
    hipStream_t st = ctx->st;
    HIPCHK(hipMemsetAsync(ctx->d_err, 0, sizeof(int), st));
    for (size_t k = 0; k < ctx->ph.size(); ++k) {
        if (!c[k]) return fail(ctx, HSW_E_INVAL, "c[k] is NULL");
        const ProbHost& h = ctx->ph[k];
        HIPCHK(hipMemcpyAsync(ctx->d_c + h.c_off, c[k], 8 * (size_t)h.Nint, hipMemcpyDeviceToDevice, st));
        launch_check_velocity(ctx->d_c + h.c_off, h.Nint, ctx->d_err, st);
        const hsw_problem& q = ctx->probs[k];
        for (int j = 0; j < 3; ++j)
            launch_axis_table(ctx->d_et + ctx->prob_h[k].e_off[j], q.n[j], q.gamma, q.h, q.pml_amp,
                              q.omega, st);
    }
    for (auto& P : ctx->pan_h) {
        const hsw_problem& q = ctx->probs[P.prob];
        launch_aux_table(ctx->d_et + P.e3_off, q.n[2], q.gamma, P.lo, P.ga, P.nz, q.h, q.pml_amp,
                         q.omega, st);
    }
    HIPCHK(hipGetLastError());
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad) return fail(ctx, HSW_E_INVAL, "velocity must be positive and finite");
    ctx->assembled = true;
    ctx->factored = false;
    return HSW_OK;
}

template <typename T>
static hsw_status setup_impl(hsw_ctx* ctx) {
    hipStream_t st = ctx->st;
    Cx<T>* L = (Cx<T>*)ctx->d_L;
    Cx<T>* G = (Cx<T>*)ctx->d_G;
    Cx<T>* dinv = (Cx<T>*)ctx->d_dinv;
    Cx<T>* ws[2] = {(Cx<T>*)ctx->d_ws[0], (Cx<T>*)ctx->d_ws[1]};
    HIPCHK(hipMemsetAsync(ctx->d_err, 0xff, 2 * sizeof(int), st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    for (int d = ctx->maxdepth; d >= 0; --d) {
        const DepthSchedule& ds = ctx->fsched[d];
        const double es = sizeof(Cx<T>);
        timed(ctx, "assemble", ds.assemble.count, es * ds.assemble.bytes_per_esz, 0.0, [&] {
            launch_assemble<T>(ctx->d_fwork + ds.assemble.off, ds.assemble.count, ctx->d_inst,
                               ctx->d_pan, ctx->d_prob, ctx->d_perm, ctx->d_ulist, ctx->d_cmap,
                               ctx->d_et, L, ws[d & 1], ws[(d + 1) & 1], st);
        });
        // complex BF16 Schur-update inputs: on the BF16 matrix cores (1), or
        // rounded and multiplied on the FP32 ones (2, option bf16_mfma 0)
        const int bf16 = ctx->prec == HSW_C64_BF16GEMM ? (ctx->bf16_mfma ? 1 : 2) : 0;
        const int order = ctx->update_order;
        const bool left = order == 1;
        const bool hybrid = order == 2 || (order < 0);
        for (size_t s = 0; s < ds.ldlt.size(); ++s) {
            if (left)
                timed(ctx, "trailing", ds.left[s].count, es * ds.left[s].bytes_per_esz, 8 * ds.left[s].cmac, [&] {
                    launch_update<T>(ctx->d_fwork + ds.left[s].off, ds.left[s].count, ctx->d_inst, L,
                                     ws[d & 1], ds.left[s].k, 1, bf16, st);
                });
            timed(ctx, "diag", ds.ldlt[s].count, es * ds.ldlt[s].bytes_per_esz, 8 * ds.ldlt[s].cmac, [&] {
                launch_ldlt_diag<T>(ctx->d_fwork + ds.ldlt[s].off, ds.ldlt[s].count, ctx->d_inst, L,
                                    dinv, ds.ldlt[s].k, ctx->d_err, st);
            });
            timed(ctx, "panel", ds.panel[s].count, es * ds.panel[s].bytes_per_esz, 8 * ds.panel[s].cmac, [&] {
                launch_panel_trsm<T>(ctx->d_fwork + ds.panel[s].off, ds.panel[s].count, ctx->d_inst,
                                     L, dinv, ds.panel[s].k, st);
            });
            if (hybrid)
                timed(ctx, "trailing", ds.pivots[s].count, es * ds.pivots[s].bytes_per_esz, 8 * ds.pivots[s].cmac, [&] {
                    launch_update<T>(ctx->d_fwork + ds.pivots[s].off, ds.pivots[s].count, ctx->d_inst, L,
                                     ws[d & 1], ds.pivots[s].k, 3, bf16, st);
                });
            else if (!left)
                timed(ctx, "trailing", ds.trail[s].count, es * ds.trail[s].bytes_per_esz, 8 * ds.trail[s].cmac, [&] {
                    launch_update<T>(ctx->d_fwork + ds.trail[s].off, ds.trail[s].count, ctx->d_inst, L,
                                     ws[d & 1], ds.trail[s].k, 0, bf16, st);
                });
        }
        if (left || hybrid)
            timed(ctx, "schur", ds.schur.count, es * ds.schur.bytes_per_esz, 8 * ds.schur.cmac, [&] {
                launch_update<T>(ctx->d_fwork + ds.schur.off, ds.schur.count, ctx->d_inst, L, ws[d & 1],
                                 0, 2, bf16, st);
            });
    }
    // selective inversion depth by depth: in place, the rows of F_BL L_F^{-1}
    // overwrite F_BL and the rows of L_F^{-1} go to the scratch (the other row
    // blocks of the front still read L_F) and are copied over L_F afterwards
    Cx<T>* T_ = ctx->keep_factors ? nullptr : (Cx<T>*)ctx->d_T;
    const int ngroups = ctx->inv_by_depth ? ctx->maxdepth + 1 : 1;
    for (int g = 0; g < ngroups; ++g) {
        const int d = ctx->maxdepth - g;
        const Launch& il = ctx->inv_by_depth ? ctx->inv_depth[d] : ctx->inv_launch;
        const Launch& cl = ctx->inv_by_depth ? ctx->lfcopy_depth[d] : ctx->lfcopy_all;
        timed(ctx, "inverse", il.count, sizeof(Cx<T>) * il.bytes_per_esz, 8 * il.cmac, [&] {
            launch_inverse<T>(ctx->d_fwork + il.off, il.count, ctx->d_inst, L, G, T_, st);
        });
        if (T_)
            timed(ctx, "inverse", cl.count, sizeof(Cx<T>) * cl.bytes_per_esz, 0.0, [&] {
                launch_lf_copy<T>(ctx->d_fwork + cl.off, cl.count, ctx->d_inst, L, T_, st);
            });
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(e1, st));
    int err[2];
    HIPCHK(hipMemcpyAsync(err, ctx->d_err, sizeof err, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->t_setup = ms * 1e-3;
    ctx->bad_inst = err[0];
    ctx->bad_pivot = err[1];
    if (err[0] >= 0) {
        const FrontInst& f = ctx->inst_h[err[0]];
        const PanelDev& P = ctx->pan_h[f.panel];
        char buf[200];
        snprintf(buf, sizeof buf, "zero or non-finite pivot: problem %d panel %d front %d pivot %d",
                 P.prob, f.panel - ctx->ph[P.prob].panel_base, err[0] - P.inst_base, err[1]);
        ctx->factored = false;
        return fail(ctx, HSW_E_BREAKDOWN, buf);
    }
    ctx->factored = true;
    return HSW_OK;
}

extern "C" hsw_status hsw_setup(hsw_ctx* ctx) {
    if (!ctx) return HSW_E_INVAL;
    if (!ctx->assembled) return fail(ctx, HSW_E_STATE, "setup before assemble");
    return ctx->prec == HSW_C128 ? setup_impl<double>(ctx) : setup_impl<float>(ctx);
}

// ---------------------------------------------------------------------------
template <typename T>
static hsw_status ensure_mm_ws(hsw_ctx* ctx, Lane& L, int groups);

template <typename T>
static hsw_status ensure_solve_ws(hsw_ctx* ctx, Lane& L, int nrhs) {
    if (nrhs >= ctx->mm_min_rhs) {
        hsw_status s = ensure_mm_ws<T>(ctx, L, (nrhs + 15) / 16);
        if (s != HSW_OK) return s;
    }
    if (nrhs <= L.nrhs_cap) return HSW_OK;
    HIPCHK(hipStreamSynchronize(L.st));
    if (&L == &ctx->lanes[0]) drop_graphs(ctx);  // they hold the old workspace addresses
    for (void** p : {&L.d_xmid, &L.d_xu, &L.d_c2}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    const size_t e = sizeof(Cx<T>) * (size_t)nrhs;
    HIPCHK(hipMalloc(&L.d_xmid, e * (size_t)ctx->max_naux));
    HIPCHK(hipMalloc(&L.d_xu, e * (size_t)std::max<int64_t>(ctx->max_wsize, 1)));
    HIPCHK(hipMalloc(&L.d_c2, e * (size_t)std::max<int64_t>(ctx->max_c2, 1)));
    L.nrhs_cap = nrhs;
    return HSW_OK;
}

// Workspace of the matrix-core passes for `groups` groups of 16 right-hand
// sides.  The child-contribution and right-hand-side regions start zeroed:
// entries no child writes, and the auxiliary-plane entries of the right-hand
// side, are read as zeros by the passes and never written.
template <typename T>
static hsw_status ensure_mm_ws(hsw_ctx* ctx, Lane& L, int groups) {
    if (groups <= L.mm_groups) return HSW_OK;
    HIPCHK(hipStreamSynchronize(L.st));
    if (&L == &ctx->lanes[0]) drop_graphs(ctx);  // they hold the old workspace addresses
    for (void** p : {&L.d_mxu, &L.d_mc2, &L.d_mh2, &L.d_mpart}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    L.mm_groups = 0;
    const size_t e = sizeof(Cx<T>) * 16 * (size_t)groups;
    const size_t bc2 = e * (size_t)std::max<int64_t>(ctx->total_c2, 1);
    const size_t bh2 = e * (size_t)std::max<int64_t>(ctx->total_naux, 1);
    // partial blocks, in units of 1024 entries: the largest (items x splits)
    // of any depth's launch, 1024 entries per item, group and split for the
    // 64-row or 64-column items, 256 for the 16-row or 16-column ones
    int64_t parts = 1;
    for (const auto& lv : ctx->slevels)
        for (const SolveLevel& sl : lv) {
            for (int cnt : {sl.fcount[0], sl.bcount[MM_BWD_SHAPE64]})
                parts = std::max<int64_t>(parts, (int64_t)cnt * groups * mm_split(cnt, groups));
            for (int cnt : {sl.fcount[1], sl.bcount[MM_BWD_SHAPE]})
                parts = std::max<int64_t>(parts, ((int64_t)cnt * groups * mm_split(cnt, groups) + 3) / 4);
        }
    HIPCHK(hipMalloc(&L.d_mxu, e * (size_t)std::max<int64_t>(ctx->max_wsize, 1)));
    HIPCHK(hipMalloc(&L.d_mc2, bc2));
    HIPCHK(hipMalloc(&L.d_mh2, bh2));
    HIPCHK(hipMalloc(&L.d_mpart, sizeof(Cx<T>) * 1024 * (size_t)parts));
    HIPCHK(hipMemsetAsync(L.d_mc2, 0, bc2, L.st));
    HIPCHK(hipMemsetAsync(L.d_mh2, 0, bh2, L.st));
    L.mm_groups = groups;
    return HSW_OK;
}

// T_i applied to a right-hand side read from the padded grid `src` (mode 0:
// the panel's planes, zero-extended; mode 1: J_{i+1,i}^T of the next plane),
// the result written to the panel's planes of `dst` (emode 0: stored, and
// with `couple` also J_{i+1,i} applied to the next plane; emode 1: subtracted).
// Plane `plane0` of the padded grid sits at offset 0 of src and dst.
// force_f / force_b >= 0 run every depth with that block shape, and `ev`
// (two events per launch, forward launches first) times each launch: both
// serve the autotuner.
// The triangular passes read the factors, which exist next to G only when
// they are kept (a separate G block).
static bool tri_available(const hsw_ctx* ctx) {
    return ctx->tri_mode != 0 && ctx->keep_factors && ctx->d_G != ctx->d_L;
}

// The row-split forward form stages up to 64 KB of LDS per workgroup.
template <typename T>
static bool fwd_rs_fits(int smax) {
    return fwd_rs_lds_bytes<T>(smax) <= 65536;
}

template <typename T>
static void panel_tsolve(hsw_ctx* ctx, Lane& ln, int gpanel, int gmode, const Cx<double>* src,
                         int64_t ld, int plane0, int emode, int couple, Cx<double>* dst, int nrhs,
                         int force_f = -1, int force_b = -1, hipEvent_t* ev = nullptr, int mm_force_f = -1,
                         int mm_force_b = -1, bool no_mm = false) {
    hipStream_t st = ln.st;
    const PanelDev& P = ctx->pan_h[gpanel];
    const ProbDev& Q = ctx->prob_h[P.prob];
    const PanelClass& c = ctx->classes[P.cls];
    const FrontInst& f0 = ctx->inst_h[P.inst_base];
    PassArgs<T> A{};
    A.run = ln.run;
    A.G = (const Cx<T>*)ctx->d_G + f0.loff;
    A.dinv = (const Cx<T>*)ctx->d_dinv + f0.doff;
    A.cmap = ctx->d_cmap;
    A.pmap = ctx->d_pmap;
    A.hmap = ctx->d_hmap;
    A.et = ctx->d_et;
    A.src = src;
    A.dst = dst;
    A.ld = ld;
    A.xmid = (Cx<T>*)ln.d_xmid;
    A.c2 = (Cx<T>*)ln.d_c2;
    A.xu = (Cx<T>*)ln.d_xu;
    A.naux = c.naux;
    A.c2ld = (int)std::max<int64_t>(c.c2size, 1);
    A.xuld = (int)std::max<int64_t>(c.wsize, 1);
    A.nrhs = nrhs;
    A.couple = couple;
    A.plane0 = plane0;
    A.Nx = P.Nx;
    A.NxNy = P.Nx * P.Ny;
    A.nz = P.nz;
    A.ga = P.ga;
    A.lo = P.lo;
    A.hi = P.hi;
    A.e1 = Q.e_off[0];
    A.e2 = Q.e_off[1];
    A.ie3hi = Q.e_off[2] + Q.N[2] + P.hi;
    A.inv_h2 = 1.0 / (Q.h * Q.h);
    const auto& lv = ctx->slevels[P.cls];
    const double es = sizeof(Cx<T>);
    const int key = rhs_key(nrhs);
    // G entries the passes need: leaves from their first live pivot's plane
    // (forward) or from their first plane of the panel's own (backward)
    const int pf = gmode == 0 ? P.ga : P.nz - 1, pb = P.ga;
    int li = 0;
    auto run = [&](const char* cls, int count, double bytes, double flops, auto&& launch) {
        if (ev) {
            LaunchTiming& lt = launch_timing();
            lt.start = ev[2 * li];
            lt.stop = ev[2 * li + 1];
            launch();
            lt.start = lt.stop = nullptr;
        } else {
            timed(ctx, cls, count, bytes, flops, launch);
        }
        ++li;
    };
    const bool tri_ok = tri_available(ctx);
    const bool tri_all = tri_ok && ctx->tri_mode == 1;
    // the same arguments with the kept factor block in place of G
    PassArgs<T> AT = A;
    AT.G = (const Cx<T>*)ctx->d_L + f0.loff;
    if (nrhs >= ctx->mm_min_rhs && !no_mm && force_f < 0 && !tri_all) {  // matrix-core passes, 16 right-hand sides per group
        const int64_t cls_c2 = ctx->cls_c2_base[P.cls], cls_h2 = ctx->cls_perm_off[P.cls];
        A.xmid = nullptr;  // x_S sits in front of x_U, in xu
        A.xu = (Cx<T>*)ln.d_mxu;
        A.c2 = (Cx<T>*)ln.d_mc2 + 16 * cls_c2;
        A.h2 = (Cx<T>*)ln.d_mh2 + 16 * cls_h2;
        A.part = (Cx<T>*)ln.d_mpart;
        A.perm = ctx->d_perm + P.perm_off;
        A.gs_u = 16 * std::max<int64_t>(ctx->max_wsize, 1);
        A.gs_c2 = 16 * std::max<int64_t>(ctx->total_c2, 1);
        A.gs_h2 = 16 * std::max<int64_t>(ctx->total_naux, 1);
        A.mode = gmode;
        // the right-hand side in elimination order: read the panel planes (or
        // the next plane) once, write 16 right-hand sides per entry (untimed
        // while the autotuner times the passes)
        if (ev)
            launch_rhs_scatter<T>(A, st);
        else
            run("scatter", 1, (double)c.naux * ((nrhs + 15) / 16) * 16 * es +
                                  16.0 * nrhs * P.Nx * P.Ny * (gmode == 0 ? P.hi - P.lo : 1),
                0.0, [&] { launch_rhs_scatter<T>(A, st); });
        const int groups = (nrhs + 15) / 16;
        for (int d = c.maxdepth; d >= 0; --d) {
            // the form: forced, tuned, or the default rule (64-row items
            // unless they give few workgroups, complex128 16-row ones; 8
            // waves below 512 workgroups)
            int form = mm_force_f >= 0 ? mm_force_f : ctx->mm_fwd_form >= 0 ? ctx->mm_fwd_form : lv[d].mm_f;
            if (form == 2 && !fwd_rs_fits<T>(lv[d].smax)) form = 0;
            if (form < 0) {
                const bool rt4 = sizeof(T) == 4 && lv[d].fcount[0] * groups >= MM_NARROW_BELOW;
                form = rt4 ? 0 : 1;
                if (lv[d].fcount[rt4 ? 0 : 1] * groups < MM_WIDE_BELOW) form += 3;
            }
            const int fs = (form == 1 || form == 4 || form >= 6) ? 1 : 0;  // items of 16 rows
            A.items = ctx->d_sitems + lv[d].foff[fs];
            A.nsplit = mm_split(lv[d].fcount[fs], groups);
            run("fwd", lv[d].fcount[fs], es * lv[d].g_need(pf) * groups + nrhs * lv[d].fwd_vec[pf],
                8.0 * nrhs * lv[d].g_need(pf),
                [&] { launch_fwd_mm<T>(A, lv[d].fcount[fs], form, lv[d].smax, st); });
        }
        A.mode = emode;
        for (int d = 0; d <= c.maxdepth; ++d) {
            // the form: forced, tuned, or the default rule (64-column items
            // where they give enough workgroups, else 16-column ones, with 16
            // waves (complex64) below 512 workgroups)
            int form = mm_force_b >= 0 ? mm_force_b : ctx->mm_bwd_form >= 0 ? ctx->mm_bwd_form : lv[d].mm_b;
            if (form < 0) {
                if (lv[d].bcount[MM_BWD_SHAPE64] * groups >= MM_TILES4_FROM)
                    form = 0;
                else
                    form = sizeof(T) == 4 && lv[d].bcount[MM_BWD_SHAPE] * groups < MM_WIDE_BELOW ? 3 : 1;
            }
            const int bs = (form == 0 || form == 4) ? MM_BWD_SHAPE64 : MM_BWD_SHAPE;
            A.items = ctx->d_sitems + lv[d].boff[bs];
            A.nsplit = mm_split(lv[d].bcount[bs], groups);
            run("bwd", lv[d].bcount[bs], es * lv[d].g_need(pb) * groups + nrhs * lv[d].bwd_vec[pb],
                8.0 * nrhs * lv[d].g_need(pb), [&] { launch_bwd_mm<T>(A, lv[d].bcount[bs], form, st); });
        }
        return;
    }
    A.mode = AT.mode = gmode;
    for (int d = c.maxdepth; d >= 0; --d) {
        int k = force_f >= 0 ? force_f : (tri_all ? TRI_F : lv[d].fsel[key]);
        if (k == TRI_F && !tri_ok) k = lv[d].nmax >= SOLVE_SMALL_BLOCK_N ? 1 : 0;
        if (k == TRI_F) {
            AT.items = ctx->d_sitems + lv[d].toff;
            run("fwd", lv[d].tcount, es * lv[d].g_need(pf) + nrhs * lv[d].fwd_vec[pf],
                8.0 * nrhs * lv[d].g_need(pf), [&] { launch_tri<T>(AT, lv[d].tcount, lv[d].nmax, true, st); });
            continue;
        }
        A.items = ctx->d_sitems + lv[d].foff[k];
        run("fwd", lv[d].fcount[k], es * lv[d].g_need(pf) + nrhs * lv[d].fwd_vec[pf],
            8.0 * nrhs * lv[d].g_need(pf),
            [&] { launch_fwd<T>(A, lv[d].fcount[k], k, lv[d].smax, lv[d].nmax, st); });
    }
    A.mode = AT.mode = emode;
    for (int d = 0; d <= c.maxdepth; ++d) {
        int k = force_b >= 0 ? force_b : (tri_all ? TRI_B : lv[d].bsel[key]);
        if (k == TRI_B && !tri_ok) k = lv[d].nmax >= SOLVE_SMALL_BLOCK_N ? 1 : 0;
        if (k == TRI_B) {
            AT.items = ctx->d_sitems + lv[d].toff;
            run("bwd", lv[d].tcount, es * lv[d].g_need(pb) + nrhs * lv[d].bwd_vec[pb],
                8.0 * nrhs * lv[d].g_need(pb), [&] { launch_tri<T>(AT, lv[d].tcount, lv[d].nmax, false, st); });
            continue;
        }
        A.items = ctx->d_sitems + lv[d].boff[k];
        run("bwd", lv[d].bcount[k], es * lv[d].g_need(pb) + nrhs * lv[d].bwd_vec[pb],
            8.0 * nrhs * lv[d].g_need(pb),
            [&] { launch_bwd<T>(A, lv[d].bcount[k], k, lv[d].nmax, st); });
    }
}

// Autotuner of the solve passes: for every panel class and tree depth, time
// each block shape of the forward and the backward pass inside whole panel
// solves (cycling over the class's panels, so the factors are not cache
// resident more than in a sweep) and keep the fastest, per right-hand-side
// group.  Runs once per group, at the first solve after a setup; the plan
// and the factors' values do not affect the choice.
template <typename T>
static hsw_status tune_solve_mm(hsw_ctx* ctx);

template <typename T>
static hsw_status tune_solve(hsw_ctx* ctx, int nrhs) {
    const int key = rhs_key(nrhs);
    if (nrhs >= ctx->mm_min_rhs) return tune_solve_mm<T>(ctx);
    // inside a multi-lane solve the shapes are fixed (tuning runs on lane 0 before it)
    if (!ctx->autotune || ctx->tuned[key] || ctx->in_lanes) return HSW_OK;
    constexpr int REPS = 3;
    // candidates: every block shape, plus the triangular passes when the factors are kept
    const bool tri = tri_available(ctx);
    const int NS = std::max(N_FWD_SHAPES, N_BWD_SHAPES) + (tri ? 1 : 0);
    int64_t plen = 1;
    for (const PanelDev& P : ctx->pan_h) plen = std::max<int64_t>(plen, (int64_t)(P.hi - P.lo) * P.Nx * P.Ny);
    Cx<double>* v = nullptr;
    const int nl = 2 * (ctx->maxdepth + 1);
    std::vector<hipEvent_t> ev(2 * nl, nullptr);
    hsw_status status = HSW_OK;
    auto cleanup = [&] {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (v) (void)hipFree(v);
    };
#define TCHK(expr)                                                         \
    do {                                                                   \
        hipError_t e_ = (expr);                                            \
        if (e_ != hipSuccess) {                                            \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);  \
            cleanup();                                                     \
            return HSW_E_DEVICE;                                           \
        }                                                                  \
    } while (0)
    TCHK(hipMalloc(&v, 16 * (size_t)plen * nrhs));
    TCHK(hipMemsetAsync(v, 0, 16 * (size_t)plen * nrhs, ctx->st));
    for (hipEvent_t& e : ev) TCHK(hipEventCreate(&e));
    for (size_t ci = 0; ci < ctx->classes.size(); ++ci) {
        const PanelClass& c = ctx->classes[ci];
        std::vector<int> panels;
        for (size_t g = 0; g < ctx->pan_h.size(); ++g)
            if (ctx->pan_h[g].cls == (int)ci) panels.push_back((int)g);
        const int D = c.maxdepth;
        std::vector<std::vector<float>> tf(D + 1, std::vector<float>(N_FWD_SHAPES + 1, 1e30f));
        std::vector<std::vector<float>> tb(D + 1, std::vector<float>(N_BWD_SHAPES + 1, 1e30f));
        int run = 0;
        for (int rep = 0; rep < REPS; ++rep)
            for (int k = 0; k < NS; ++k, ++run) {
                const int gp = panels[run % panels.size()];
                const bool kt = tri && k == NS - 1;
                const int kf = kt ? TRI_F : k % N_FWD_SHAPES, kb = kt ? TRI_B : k % N_BWD_SHAPES;
                const PanelDev& P = ctx->pan_h[gp];
                panel_tsolve<T>(ctx, ctx->lanes[0], gp, 0, v, plen, P.lo, 0, 0, v, nrhs, kf, kb, ev.data());
                TCHK(hipGetLastError());
                TCHK(hipEventSynchronize(ev[2 * (2 * (D + 1)) - 1]));
                for (int l = 0; l < 2 * (D + 1); ++l) {
                    float ms = 0;
                    TCHK(hipEventElapsedTime(&ms, ev[2 * l], ev[2 * l + 1]));
                    if (l <= D) {
                        const int d = D - l;
                        tf[d][kf] = std::min(tf[d][kf], ms);
                    } else {
                        const int d = l - (D + 1);
                        tb[d][kb] = std::min(tb[d][kb], ms);
                    }
                }
            }
        for (int d = 0; d <= D; ++d) {
            SolveLevel& sl = ctx->slevels[ci][d];
            sl.fsel[key] = (int)(std::min_element(tf[d].begin(), tf[d].end()) - tf[d].begin());
            sl.bsel[key] = (int)(std::min_element(tb[d].begin(), tb[d].end()) - tb[d].begin());
        }
    }
#undef TCHK
    cleanup();
    ctx->tuned[key] = true;
    return status;
}

// Autotuner of the matrix-core passes: for every panel class and tree depth,
// time items of 64 and of 16 rows and the row-split form (forward) and items
// of 64 and of 16 columns (backward) inside whole panel solves of one group of
// 16 right-hand sides, cycling over the class's panels, and keep the fastest
// of each.  Runs once, at the first solve with 16 or more right-hand sides
// after a setup.
template <typename T>
static hsw_status tune_solve_mm(hsw_ctx* ctx) {
    if (!ctx->autotune || ctx->tuned_mm || ctx->in_lanes) return HSW_OK;
    constexpr int REPS = 3, NR = MM_MIN_RHS;
    hsw_status st = ensure_solve_ws<T>(ctx, ctx->lanes[0], NR);
    if (st != HSW_OK) return st;
    int64_t plen = 1;
    for (const PanelDev& P : ctx->pan_h) plen = std::max<int64_t>(plen, (int64_t)(P.hi - P.lo) * P.Nx * P.Ny);
    Cx<double>* v = nullptr;
    const int nl = 2 * (ctx->maxdepth + 1);
    std::vector<hipEvent_t> ev(2 * nl, nullptr);
    auto cleanup = [&] {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (v) (void)hipFree(v);
    };
#define TCHK(expr)                                                         \
    do {                                                                   \
        hipError_t e_ = (expr);                                            \
        if (e_ != hipSuccess) {                                            \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);  \
            cleanup();                                                     \
            return HSW_E_DEVICE;                                           \
        }                                                                  \
    } while (0)
    TCHK(hipMalloc(&v, 16 * (size_t)plen * NR));
    TCHK(hipMemsetAsync(v, 0, 16 * (size_t)plen * NR, ctx->st));
    for (hipEvent_t& e : ev) TCHK(hipEventCreate(&e));
    for (size_t ci = 0; ci < ctx->classes.size(); ++ci) {
        const PanelClass& c = ctx->classes[ci];
        std::vector<int> panels;
        for (size_t g = 0; g < ctx->pan_h.size(); ++g)
            if (ctx->pan_h[g].cls == (int)ci) panels.push_back((int)g);
        const int D = c.maxdepth;
        constexpr int NF = 8, NB = 9;  // forward and backward forms
        constexpr int NK = NF > NB ? NF : NB;
        std::vector<std::array<float, NF>> tf(D + 1);
        std::vector<std::array<float, NB>> tb(D + 1);
        for (auto& a : tf) a.fill(1e30f);
        for (auto& a : tb) a.fill(1e30f);
        int run = 0;
        for (int rep = 0; rep < REPS; ++rep)
            for (int k = 0; k < NK; ++k, ++run) {
                const int gp = panels[run % panels.size()];
                const PanelDev& P = ctx->pan_h[gp];
                // forward form min(k, NF - 1) and backward form min(k, NB - 1) at every depth
                panel_tsolve<T>(ctx, ctx->lanes[0], gp, 0, v, plen, P.lo, 0, 0, v, NR, -1, -1, ev.data(),
                                std::min(k, NF - 1), std::min(k, NB - 1));
                TCHK(hipGetLastError());
                TCHK(hipEventSynchronize(ev[2 * (2 * (D + 1)) - 1]));
                for (int l = 0; l < 2 * (D + 1); ++l) {
                    float ms = 0;
                    TCHK(hipEventElapsedTime(&ms, ev[2 * l], ev[2 * l + 1]));
                    if (l <= D) {
                        float& t = tf[D - l][std::min(k, NF - 1)];
                        t = std::min(t, ms);
                    } else {
                        float& t = tb[l - (D + 1)][std::min(k, NB - 1)];
                        t = std::min(t, ms);
                    }
                }
            }
        for (int d = 0; d <= D; ++d) {
            SolveLevel& sl = ctx->slevels[ci][d];
            if (!fwd_rs_fits<T>(sl.smax)) tf[d][2] = 1e30f;  // ran as form 0
            sl.mm_f = 0;
            for (int k = 1; k < NF; ++k)
                if (tf[d][k] < tf[d][sl.mm_f]) sl.mm_f = k;
            sl.mm_b = 0;
            for (int k = 1; k < NB; ++k)
                if (tb[d][k] < tb[d][sl.mm_b]) sl.mm_b = k;
            if (ctx->tune_report) {
                // algorithmic bytes of each pass at this depth (as the pass timers count them)
                const int ga = ctx->pan_h[panels[panels.size() / 2]].ga;  // a middle panel's
                const double fb = ctx->esz * sl.g_need(ga) + NR * sl.fwd_vec[ga];
                const double bb = ctx->esz * sl.g_need(ga) + NR * sl.bwd_vec[ga];
                fprintf(stderr, "tune class %zu depth %d fronts %zu fwd", ci, d, c.at_depth[d].size());
                for (int k = 0; k < NF; ++k) fprintf(stderr, " %.1f", 1e3 * tf[d][k]);
                fprintf(stderr, " -> %d (%.1f MB, %.2f TB/s)  bwd", sl.mm_f, fb / 1e6,
                        fb / (1e9 * tf[d][sl.mm_f]));
                for (int k = 0; k < NB; ++k) fprintf(stderr, " %.1f", 1e3 * tb[d][k]);
                fprintf(stderr, " -> %d (%.1f MB, %.2f TB/s) (us)\n", sl.mm_b, bb / 1e6, bb / (1e9 * tb[d][sl.mm_b]));
            }
        }
    }
#undef TCHK
    cleanup();
    ctx->tuned_mm = true;
    return HSW_OK;
}

// z := M^{-1} r (Alg. 1.5), r may equal z.
template <typename T>
static hsw_status sweep_impl(hsw_ctx* ctx, Lane& ln, int prob, const Cx<double>* r, Cx<double>* z,
                             int nrhs, int64_t ld) {
    hsw_status s = ensure_solve_ws<T>(ctx, ln, nrhs);
    if (s == HSW_OK) s = tune_solve<T>(ctx, nrhs);
    if (s != HSW_OK) return s;
    const ProbHost& h = ctx->ph[prob];
    if (r != z && ln.run)
        launch_copy_cols(r, z, ld, h.Npad, nrhs, ln.run, ln.st);
    else if (r != z)
        HIPCHK(hipMemcpy2DAsync(z, 16 * ld, r, 16 * ld, 16 * h.Npad, nrhs, hipMemcpyDeviceToDevice,
                                ln.st));
    for (int i = 0; i < h.m; ++i)
        panel_tsolve<T>(ctx, ln, h.panel_base + i, 0, z, ld, 0, 0, i < h.m - 1, z, nrhs);
    for (int i = h.m - 2; i >= 0; --i)
        panel_tsolve<T>(ctx, ln, h.panel_base + i, 1, z, ld, 0, 1, 0, z, nrhs);
    HIPCHK(hipGetLastError());
    return HSW_OK;
}

// z := M^{-1} r through a captured sweep when graphs are enabled: r is copied
// to the graph's own vector, the graph replays the 2m - 1 panel solves of
// Alg. 1.5 on it, and the result is copied to z.  The graph runs on a
// context-owned stream joined to st by events before and after.
template <typename T>
static hsw_status sweep_any(hsw_ctx* ctx, Lane& ln, int prob, const Cx<double>* r, Cx<double>* z,
                            int nrhs, int64_t ld) {
    if (&ln != &ctx->lanes[0] || !ctx->use_graph || ctx->timer.on || ctx->in_lanes)
        return sweep_impl<T>(ctx, ln, prob, r, z, nrhs, ld);
    hsw_status s = ensure_solve_ws<T>(ctx, ln, nrhs);
    if (s == HSW_OK) s = tune_solve<T>(ctx, nrhs);
    if (s != HSW_OK) return s;
    const ProbHost& h = ctx->ph[prob];
    const int64_t N = h.Npad;
    if (!ctx->gst) {
        HIPCHK(hipStreamCreateWithFlags(&ctx->gst, hipStreamNonBlocking));
        for (hipEvent_t& e : ctx->gev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    SweepGraph* g = nullptr;
    for (SweepGraph& q : ctx->graphs)
        if (q.prob == prob && q.nrhs == nrhs && q.cycle_k == 0) g = &q;
    if (!g) {
        SweepGraph ng;
        ng.prob = prob;
        ng.nrhs = nrhs;
        HIPCHK(hipMalloc(&ng.z, 16 * (size_t)N * nrhs));
        Cx<double>* zz = (Cx<double>*)ng.z;
        Lane gl;  // lane 0's workspaces on the capture stream
        gl.st = ctx->gst;
        gl.d_xmid = ln.d_xmid;
        gl.d_xu = ln.d_xu;
        gl.d_c2 = ln.d_c2;
        gl.nrhs_cap = ln.nrhs_cap;
        gl.d_mxu = ln.d_mxu;
        gl.d_mc2 = ln.d_mc2;
        gl.d_mh2 = ln.d_mh2;
        gl.d_mpart = ln.d_mpart;
        gl.mm_groups = ln.mm_groups;
        hipError_t e = hipStreamBeginCapture(ctx->gst, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int i = 0; i < h.m; ++i)
                panel_tsolve<T>(ctx, gl, h.panel_base + i, 0, zz, N, 0, 0, i < h.m - 1, zz, nrhs);
            for (int i = h.m - 2; i >= 0; --i)
                panel_tsolve<T>(ctx, gl, h.panel_base + i, 1, zz, N, 0, 1, 0, zz, nrhs);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(ctx->gst, &graph);
            if (e == hipSuccess) e = hipGraphInstantiate(&ng.exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
        }
        if (e != hipSuccess) {
            (void)hipFree(ng.z);
            return fail(ctx, HSW_E_DEVICE, std::string("sweep capture: ") + hipGetErrorString(e));
        }
        ctx->graphs.push_back(ng);
        g = &ctx->graphs.back();
    }
    HIPCHK(hipMemcpy2DAsync(g->z, 16 * N, r, 16 * ld, 16 * N, nrhs, hipMemcpyDeviceToDevice, ctx->st));
    HIPCHK(hipEventRecord(ctx->gev[0], ctx->st));
    HIPCHK(hipStreamWaitEvent(ctx->gst, ctx->gev[0], 0));
    HIPCHK(hipGraphLaunch(g->exec, ctx->gst));
    HIPCHK(hipEventRecord(ctx->gev[1], ctx->gst));
    HIPCHK(hipStreamWaitEvent(ctx->st, ctx->gev[1], 0));
    HIPCHK(hipMemcpy2DAsync(z, 16 * ld, g->z, 16 * N, 16 * N, nrhs, hipMemcpyDeviceToDevice, ctx->st));
    return HSW_OK;
}

static hsw_status check_vec_args(hsw_ctx* ctx, int32_t prob, const void* a, const void* b,
                                 int32_t nrhs, int64_t ld, int64_t minld) {
    if (prob < 0 || prob >= (int)ctx->ph.size()) return fail(ctx, HSW_E_INVAL, "bad problem index");
    if (!a || !b) return fail(ctx, HSW_E_INVAL, "NULL vector");
    if (nrhs < 1 || ld < minld) return fail(ctx, HSW_E_INVAL, "nrhs >= 1 and ld >= vector length required");
    return HSW_OK;
}

extern "C" hsw_status hsw_apply(hsw_ctx* ctx, int32_t prob, const hsw_c128* r, hsw_c128* z,
                                int32_t nrhs, int64_t ld) {
    if (!ctx) return HSW_E_INVAL;
    if (!ctx->factored) return fail(ctx, HSW_E_STATE, "apply before setup");
    if (prob < 0 || prob >= (int)ctx->ph.size()) return fail(ctx, HSW_E_INVAL, "bad problem index");
    hsw_status s = check_vec_args(ctx, prob, r, z, nrhs, ld, ctx->ph[prob].Npad);
    if (s != HSW_OK) return s;
    if ((const void*)r == (const void*)z) return fail(ctx, HSW_E_INVAL, "r and z alias");
    return ctx->prec == HSW_C128
               ? sweep_any<double>(ctx, ctx->lanes[0], prob, (const Cx<double>*)r, (Cx<double>*)z, nrhs, ld)
               : sweep_any<float>(ctx, ctx->lanes[0], prob, (const Cx<double>*)r, (Cx<double>*)z, nrhs, ld);
}

// ---------------------------------------------------------------------------
// The allocation-free sweep: hsw_apply with the panel-solve workspace in a
// file-scope device array instead of memory the library allocates.  Each
// device the library runs on holds its own copy of the array until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device, kept per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's scratch (looked up once per device).
hipError_t scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

template <typename T>
static hsw_status apply_noalloc_impl(hsw_ctx* ctx, int prob, const Cx<double>* r, Cx<double>* z, int nrhs,
                                     int64_t ld, void* base) {
    // the lane-0 workspace layout (x_mid, update-set values, child slots) in the scratch
    const size_t e = sizeof(Cx<T>) * (size_t)nrhs;
    const size_t bx = (e * (size_t)ctx->max_naux + 255) / 256 * 256;
    const size_t bu = (e * (size_t)std::max<int64_t>(ctx->max_wsize, 1) + 255) / 256 * 256;
    const size_t bc = e * (size_t)std::max<int64_t>(ctx->max_c2, 1);
    if (bx + bu + bc > NOALLOC_SCRATCH_BYTES) {
        char buf[200];
        snprintf(buf, sizeof buf, "apply_noalloc: %d right-hand sides need %.1f MB of workspace, the scratch "
                 "holds %.1f MB", nrhs, (bx + bu + bc) / 1e6, NOALLOC_SCRATCH_BYTES / 1e6);
        return fail(ctx, HSW_E_INVAL, buf);
    }
    Lane ln;
    ln.st = ctx->st;
    ln.d_xmid = base;
    ln.d_xu = (unsigned char*)base + bx;
    ln.d_c2 = (unsigned char*)base + bx + bu;
    ln.nrhs_cap = nrhs;
    const ProbHost& h = ctx->ph[prob];
    HIPCHK(hipMemcpy2DAsync(z, 16 * ld, r, 16 * ld, 16 * h.Npad, nrhs, hipMemcpyDeviceToDevice, ctx->st));
    // the single-vector passes whatever mm_min_rhs says (the matrix-core
    // passes' workspaces are not in the scratch)
    for (int i = 0; i < h.m; ++i)
        panel_tsolve<T>(ctx, ln, h.panel_base + i, 0, z, ld, 0, 0, i < h.m - 1, z, nrhs, -1, -1, nullptr, -1, -1,
                        true);
    for (int i = h.m - 2; i >= 0; --i)
        panel_tsolve<T>(ctx, ln, h.panel_base + i, 1, z, ld, 0, 1, 0, z, nrhs, -1, -1, nullptr, -1, -1, true);
    HIPCHK(hipGetLastError());
    return HSW_OK;
}

extern "C" hsw_status hsw_apply_noalloc(hsw_ctx* ctx, int32_t prob, const hsw_c128* r, hsw_c128* z,
                                        int32_t nrhs, int64_t ld) {
    if (!ctx) return HSW_E_INVAL;
    if (!ctx->factored) return fail(ctx, HSW_E_STATE, "apply before setup");
    hsw_status s = check_vec_args(ctx, prob, r, z, nrhs, ld, ctx->ph[prob >= 0 && prob < (int)ctx->ph.size() ? prob : 0].Npad);
    if (s != HSW_OK) return s;
    if ((const void*)r == (const void*)z) return fail(ctx, HSW_E_INVAL, "r and z alias");
    if (nrhs >= MM_MIN_RHS)
        return fail(ctx, HSW_E_INVAL, "apply_noalloc takes at most 15 right-hand sides per call");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != ctx->device || dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(ctx, HSW_E_INVAL, "apply_noalloc: make the context's device current");
    void* base = nullptr;
    HIPCHK(scratch_address(dev, &base));
    return ctx->prec == HSW_C128
               ? apply_noalloc_impl<double>(ctx, prob, (const Cx<double>*)r, (Cx<double>*)z, nrhs, ld, base)
               : apply_noalloc_impl<float>(ctx, prob, (const Cx<double>*)r, (Cx<double>*)z, nrhs, ld, base);
}

extern "C" hsw_status hsw_panel_solve(hsw_ctx* ctx, int32_t prob, int32_t panel, const hsw_c128* v,
                                      hsw_c128* y, int32_t nrhs, int64_t ld) {
    if (!ctx) return HSW_E_INVAL;
    if (!ctx->factored) return fail(ctx, HSW_E_STATE, "panel solve before setup");
    if (prob < 0 || prob >= (int)ctx->ph.size()) return fail(ctx, HSW_E_INVAL, "bad problem index");
    const ProbHost& h = ctx->ph[prob];
    if (panel < 0 || panel >= h.m) return fail(ctx, HSW_E_INVAL, "bad panel index");
    const PanelDev& P = ctx->pan_h[h.panel_base + panel];
    hsw_status s = check_vec_args(ctx, prob, v, y, nrhs, ld, (int64_t)(P.hi - P.lo) * P.Nx * P.Ny);
    if (s != HSW_OK) return s;
    if ((const void*)v == (const void*)y) return fail(ctx, HSW_E_INVAL, "v and y alias");
    if (ctx->prec == HSW_C128) {
        s = ensure_solve_ws<double>(ctx, ctx->lanes[0], nrhs);
        if (s != HSW_OK) return s;
        panel_tsolve<double>(ctx, ctx->lanes[0], h.panel_base + panel, 0, (const Cx<double>*)v, ld, P.lo, 0, 0,
                             (Cx<double>*)y, nrhs);
    } else {
        s = ensure_solve_ws<float>(ctx, ctx->lanes[0], nrhs);
        if (s != HSW_OK) return s;
        panel_tsolve<float>(ctx, ctx->lanes[0], h.panel_base + panel, 0, (const Cx<double>*)v, ld, P.lo, 0, 0,
                            (Cx<double>*)y, nrhs);
    }
    HIPCHK(hipGetLastError());
    return HSW_OK;
}

extern "C" hsw_status hsw_matvec(hsw_ctx* ctx, int32_t prob, const hsw_c128* x, hsw_c128* y,
                                 int32_t nrhs, int64_t ld) {
    if (!ctx) return HSW_E_INVAL;
    if (!ctx->assembled) return fail(ctx, HSW_E_STATE, "matvec before assemble");
    if (prob < 0 || prob >= (int)ctx->ph.size()) return fail(ctx, HSW_E_INVAL, "bad problem index");
    hsw_status s = check_vec_args(ctx, prob, x, y, nrhs, ld, ctx->ph[prob].Npad);
    if (s != HSW_OK) return s;
    if ((const void*)x == (const void*)y) return fail(ctx, HSW_E_INVAL, "x and y alias");
    const double np_ = (double)ctx->ph[prob].Npad;
    timed(ctx, "matvec", 1, np_ * (32.0 * nrhs + 8.0), 56.0 * np_ * nrhs, [&] {
        launch_matvec(ctx->prob_h[prob], ctx->d_et, (const Cx<double>*)x, (Cx<double>*)y, nullptr, ld,
                      nrhs, 0, ctx->st);
    });
    HIPCHK(hipGetLastError());
    return HSW_OK;
}

// ---------------------------------------------------------------------------
// Flexible right-preconditioned GMRES(k) of one problem, all right-hand
// sides advanced together; classical Gram-Schmidt applied twice.
// The k Arnoldi steps of one GMRES cycle with the convergence test on the
// device (k_conv after each step; every kernel stops at its start once
// *run is 0).  With the option graph, on lane 0 and while no kernel class
// is timed, the steps are captured once per (problem, right-hand-side
// count, k) and replayed.
template <typename T>
static hsw_status gmres_cycle_device(hsw_ctx* ctx, Lane& ln, int prob, Cx<double>* V, Cx<double>* Z,
                                     Cx<double>* H, Cx<double>* part, Cx<double>* coef, double* cs,
                                     Cx<double>* sn, Cx<double>* g, const double* bn, double* est, double* nrm,
                                     double* partn, int* act, int* jc, int* itd, int* run, int nrhs, int k,
                                     const hsw_solve_opts& o) {
    const ProbDev& Q = ctx->prob_h[prob];
    const int64_t N = ctx->ph[prob].Npad, ld = N, vs = N * nrhs;
    const int hld = (k + 1) * k;
    auto steps = [&](Lane& L) -> hsw_status {
        hipStream_t st = L.st;
        L.run = run;
        for (int j = 0; j < k; ++j) {
            Cx<double>* Vj = V + (int64_t)j * vs;
            Cx<double>* Vn = V + (int64_t)(j + 1) * vs;
            Cx<double>* Zj = Z + (int64_t)j * vs;
            hsw_status s = sweep_impl<T>(ctx, L, prob, Vj, Zj, nrhs, ld);
            if (s != HSW_OK) {
                L.run = nullptr;
                return s;
            }
            timed(ctx, "matvec", 1, (double)N * (32.0 * nrhs + 8.0), 56.0 * (double)N * nrhs,
                  [&] { launch_matvec(Q, ctx->d_et, Zj, Vn, nullptr, ld, nrhs, 0, st, act, run); });
            // classical Gram-Schmidt twice: products, update fused with the second
            // products, update
            launch_dots(V, vs, Vn, ld, N, j + 1, nrhs, act, part, H + (int64_t)j * (k + 1), hld, coef, 0, st);
            launch_axpy_dots(V, vs, Vn, ld, N, j + 1, coef, hld, nrhs, act, part, H + (int64_t)j * (k + 1), hld, coef,
                             st);
            launch_axpy_multi(V, vs, Vn, ld, N, j + 1, coef, hld, nullptr, act, 0, nrhs, st);
            launch_norm(Vn, ld, N, nrhs, act, partn, nrm, H + (int64_t)j * (k + 1) + j + 1, hld, st);
            launch_scale(Vn, Vn, ld, N, nrhs, nrm, act, st);
            launch_givens(j, k, nrhs, H, cs, sn, g, bn, est, act, st);
            launch_conv(j, nrhs, est, o.rtol, o.maxit, act, itd, jc, run, st);
        }
        L.run = nullptr;
        return HSW_OK;
    };
    if (&ln != &ctx->lanes[0] || !ctx->use_graph || ctx->timer.on || ctx->in_lanes) return steps(ln);
    // workspaces and tuned shapes first: nothing may allocate or synchronise
    // during the capture
    hsw_status s = ensure_solve_ws<T>(ctx, ln, nrhs);
    if (s == HSW_OK) s = tune_solve<T>(ctx, nrhs);
    if (s != HSW_OK) return s;
    if (!ctx->gst) {
        HIPCHK(hipStreamCreateWithFlags(&ctx->gst, hipStreamNonBlocking));
        for (hipEvent_t& e : ctx->gev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    SweepGraph* gr = nullptr;
    for (SweepGraph& q : ctx->graphs)
        if (q.prob == prob && q.nrhs == nrhs && q.cycle_k == k) gr = &q;
    if (!gr) {
        SweepGraph ng;
        ng.prob = prob;
        ng.nrhs = nrhs;
        ng.cycle_k = k;
        Lane gl;  // lane 0's workspaces on the capture stream
        gl.st = ctx->gst;
        gl.d_xmid = ln.d_xmid;
        gl.d_xu = ln.d_xu;
        gl.d_c2 = ln.d_c2;
        gl.nrhs_cap = ln.nrhs_cap;
        gl.d_mxu = ln.d_mxu;
        gl.d_mc2 = ln.d_mc2;
        gl.d_mh2 = ln.d_mh2;
        gl.d_mpart = ln.d_mpart;
        gl.mm_groups = ln.mm_groups;
        hipError_t e = hipStreamBeginCapture(ctx->gst, hipStreamCaptureModeThreadLocal);
        hsw_status cs_ = HSW_OK;
        if (e == hipSuccess) {
            cs_ = steps(gl);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(ctx->gst, &graph);
            if (e == hipSuccess && cs_ == HSW_OK) e = hipGraphInstantiate(&ng.exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
        }
        if (cs_ != HSW_OK) return cs_;
        if (e != hipSuccess) return fail(ctx, HSW_E_DEVICE, std::string("cycle capture: ") + hipGetErrorString(e));
        ctx->graphs.push_back(ng);
        gr = &ctx->graphs.back();
    }
    HIPCHK(hipEventRecord(ctx->gev[0], ln.st));
    HIPCHK(hipStreamWaitEvent(ctx->gst, ctx->gev[0], 0));
    HIPCHK(hipGraphLaunch(gr->exec, ctx->gst));
    HIPCHK(hipEventRecord(ctx->gev[1], ctx->gst));
    HIPCHK(hipStreamWaitEvent(ln.st, ctx->gev[1], 0));
    return HSW_OK;
}

template <typename T>
static hsw_status gmres_impl(hsw_ctx* ctx, Lane& ln, int prob, const Cx<double>* b, Cx<double>* x,
                             int nrhs, const hsw_solve_opts& o, int* iters_out, double* relres_out) {
    hipStream_t st = ln.st;
    const ProbHost& hp = ctx->ph[prob];
    const ProbDev& Q = ctx->prob_h[prob];
    const int64_t N = hp.Npad, ld = N;
    const int k = o.restart_k;
    const int64_t vs = N * nrhs;
    const int nch = dots_chunks(N);
    const int hld = (k + 1) * k;
    Cx<double> *V = nullptr, *Z = nullptr, *H = nullptr, *coef = nullptr, *sn = nullptr, *g = nullptr,
               *y = nullptr, *part = nullptr;
    double *cs = nullptr, *bn = nullptr, *beta = nullptr, *est = nullptr, *nrm = nullptr, *partn = nullptr;
    int *act = nullptr, *jc = nullptr, *itd = nullptr, *run = nullptr;
    auto cleanup = [&]() {};  // the workspace stays with the context
#define GCHK(expr)                                                                     \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            cleanup();                                                                 \
            return fail(ctx, HSW_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                              \
    } while (0)
    {
        void** slots[] = {(void**)&V, (void**)&Z, (void**)&H, (void**)&coef, (void**)&sn, (void**)&g,
                          (void**)&y, (void**)&part, (void**)&cs, (void**)&bn, (void**)&beta,
                          (void**)&est, (void**)&nrm, (void**)&partn, (void**)&act, (void**)&jc,
                          (void**)&itd, (void**)&run};
        const size_t bytes[] = {16 * (size_t)vs * (k + 1), 16 * (size_t)vs * k, 16 * (size_t)nrhs * hld,
                                16 * (size_t)nrhs * hld, 16 * (size_t)nrhs * k, 16 * (size_t)nrhs * (k + 1),
                                16 * (size_t)nrhs * k, 16 * (size_t)nrhs * nch * (k + 1), 8 * (size_t)nrhs * k,
                                8 * (size_t)nrhs, 8 * (size_t)nrhs, 8 * (size_t)nrhs, 8 * (size_t)nrhs,
                                8 * (size_t)nrhs * nch, 4 * (size_t)nrhs, 4 * (size_t)nrhs, 4 * (size_t)nrhs, 4};
        const size_t nslot = sizeof(bytes) / sizeof(bytes[0]);
        if (ln.gws.size() < nslot) ln.gws.resize(nslot, {nullptr, 0});
        for (size_t i = 0; i < nslot; ++i) {
            auto& w = ln.gws[i];
            if (w.second < bytes[i]) {
                if (&ln == &ctx->lanes[0]) drop_graphs(ctx);  // captured cycles hold the old addresses
                if (w.first) GCHK(hipFree(w.first));
                w = {nullptr, 0};
                GCHK(hipMalloc(&w.first, bytes[i]));
                w.second = bytes[i];
            }
            *slots[i] = w.first;
        }
    }
    hsw_status s = ensure_solve_ws<T>(ctx, ln, nrhs);
    if (s != HSW_OK) { cleanup(); return s; }
    std::vector<double> bn_h(nrhs), beta_h(nrhs), est_h(nrhs), rel(nrhs, 1.0);
    std::vector<int> act_h(nrhs), it_h(nrhs, 0), jc_h(nrhs), done(nrhs, 0);
    GCHK(hipMemsetAsync(H, 0, 16 * (size_t)nrhs * hld, st));
    GCHK(hipMemset2DAsync(x, 16 * ld, 0, 16 * N, nrhs, st));
    launch_norm(b, ld, N, nrhs, nullptr, partn, bn, nullptr, 0, st);
    GCHK(hipMemcpyAsync(bn_h.data(), bn, 8 * nrhs, hipMemcpyDeviceToHost, st));
    GCHK(hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; ++r) {
        done[r] = !(bn_h[r] > 0);
        if (done[r]) rel[r] = 0.0;
    }
    // With the test on the device (option gmres_device_test), the steps of a
    // cycle are issued without reading anything back: k_conv counts each
    // step and clears act[r] when a right-hand side converges, and once all
    // have, the run flag stops every later kernel of the cycle at its start.
    // The iteration counts come back with the next cycle's residual norms,
    // so a cycle costs one read.  The cycle's steps can then be captured
    // once and replayed (option graph, on the context's own lane).
    const bool dev = ctx->gmres_device_test;
    bool first = true;
    while (true) {
        // true residual r = b - A x into V_0
        launch_matvec(Q, ctx->d_et, x, V, b, ld, nrhs, 1, st);
        launch_norm(V, ld, N, nrhs, nullptr, partn, beta, nullptr, 0, st);
        GCHK(hipMemcpyAsync(beta_h.data(), beta, 8 * nrhs, hipMemcpyDeviceToHost, st));
        if (dev && !first) GCHK(hipMemcpyAsync(it_h.data(), itd, 4 * nrhs, hipMemcpyDeviceToHost, st));
        GCHK(hipStreamSynchronize(st));
        first = false;
        bool any = false;
        for (int r = 0; r < nrhs; ++r) {
            if (!(bn_h[r] > 0)) { act_h[r] = 0; continue; }
            rel[r] = beta_h[r] / bn_h[r];
            if (rel[r] < o.rtol || it_h[r] >= o.maxit) done[r] = 1;
            act_h[r] = !done[r];
            any = any || act_h[r];
        }
        if (!any) break;
        GCHK(hipMemcpyAsync(act, act_h.data(), 4 * nrhs, hipMemcpyHostToDevice, st));
        launch_scale(V, V, ld, N, nrhs, beta, act, st);
        launch_cycle_init(k, nrhs, beta, g, act, st);
        std::fill(jc_h.begin(), jc_h.end(), 0);
        if (dev) {
            const int one = 1;
            GCHK(hipMemcpyAsync(itd, it_h.data(), 4 * nrhs, hipMemcpyHostToDevice, st));
            GCHK(hipMemcpyAsync(jc, jc_h.data(), 4 * nrhs, hipMemcpyHostToDevice, st));
            GCHK(hipMemcpyAsync(run, &one, 4, hipMemcpyHostToDevice, st));
            s = gmres_cycle_device<T>(ctx, ln, prob, V, Z, H, part, coef, cs, sn, g, bn, est, nrm, partn,
                                      act, jc, itd, run, nrhs, k, o);
            if (s != HSW_OK) { cleanup(); return s; }
            launch_lsq(k, nrhs, H, g, jc, y, st);
            launch_axpy_multi(Z, vs, x, ld, N, k, y, k, jc, nullptr, 1, nrhs, st);
            GCHK(hipGetLastError());
            continue;
        }
        for (int j = 0; j < k; ++j) {
            Cx<double>* Vj = V + (int64_t)j * vs;
            Cx<double>* Vn = V + (int64_t)(j + 1) * vs;
            Cx<double>* Zj = Z + (int64_t)j * vs;
            s = sweep_any<T>(ctx, ln, prob, Vj, Zj, nrhs, ld);
            if (s != HSW_OK) { cleanup(); return s; }
            timed(ctx, "matvec", 1, (double)N * (32.0 * nrhs + 8.0), 56.0 * (double)N * nrhs,
                  [&] { launch_matvec(Q, ctx->d_et, Zj, Vn, nullptr, ld, nrhs, 0, st); });
            // classical Gram-Schmidt twice: products, update fused with the second
            // products, update
            launch_dots(V, vs, Vn, ld, N, j + 1, nrhs, act, part, H + (int64_t)j * (k + 1), hld, coef, 0, st);
            launch_axpy_dots(V, vs, Vn, ld, N, j + 1, coef, hld, nrhs, act, part, H + (int64_t)j * (k + 1), hld, coef,
                             st);
            launch_axpy_multi(V, vs, Vn, ld, N, j + 1, coef, hld, nullptr, act, 0, nrhs, st);
            launch_norm(Vn, ld, N, nrhs, act, partn, nrm, H + (int64_t)j * (k + 1) + j + 1, hld, st);
            launch_scale(Vn, Vn, ld, N, nrhs, nrm, act, st);
            launch_givens(j, k, nrhs, H, cs, sn, g, bn, est, act, st);
            GCHK(hipGetLastError());
            GCHK(hipMemcpyAsync(est_h.data(), est, 8 * nrhs, hipMemcpyDeviceToHost, st));
            GCHK(hipStreamSynchronize(st));
            bool still = false;
            for (int r = 0; r < nrhs; ++r) {
                if (!act_h[r]) continue;
                it_h[r] += 1;
                jc_h[r] = j + 1;
                if (est_h[r] < o.rtol || it_h[r] >= o.maxit) act_h[r] = 0;
                still = still || act_h[r];
            }
            if (!still) break;
            GCHK(hipMemcpyAsync(act, act_h.data(), 4 * nrhs, hipMemcpyHostToDevice, st));
        }
        GCHK(hipMemcpyAsync(jc, jc_h.data(), 4 * nrhs, hipMemcpyHostToDevice, st));
        launch_lsq(k, nrhs, H, g, jc, y, st);
        launch_axpy_multi(Z, vs, x, ld, N, k, y, k, jc, nullptr, 1, nrhs, st);
        GCHK(hipGetLastError());
    }
    bool ok = true;
    for (int r = 0; r < nrhs; ++r) {
        if (iters_out) iters_out[r] = it_h[r];
        if (relres_out) relres_out[r] = rel[r];
        ok = ok && rel[r] < o.rtol;
    }
    cleanup();
#undef GCHK
    return ok ? HSW_OK : HSW_E_NOCONV;
}

// ---------------------------------------------------------------------------
// Block flexible GMRES(k) (Sec. 2.4 names block variants of GMRES as a way to
// lower the iteration count): the right-hand sides of one group (at most
// BLOCK_KRYLOV_MAX) share one block Krylov space.  Each step applies the
// sweep to the whole block, orthogonalises the new block against the basis
// by block classical Gram-Schmidt applied twice (C = V^H W on the matrix
// cores, W -= V C), and orthonormalises it by Cholesky QR applied twice
// (W^H W = S^H S, W := W S^{-1}).  The small block least-squares problem is
// reduced by complex Givens rotations on the host, which gives every
// column's residual estimate after every step.  Columns whose true relative
// residual is below rtol leave the block at a restart.
namespace {
using zc = std::complex<double>;

// G = S^H S for a q x q Hermitian G (row-major); S upper triangular
// (row-major).  Returns false if a pivot is not positive.
bool chol_upper(const std::vector<zc>& G, int q, std::vector<zc>& S) {
    S.assign((size_t)q * q, zc(0, 0));
    for (int i = 0; i < q; ++i) {
        double d = G[(size_t)i * q + i].real();
        for (int k = 0; k < i; ++k) d -= std::norm(S[(size_t)k * q + i]);
        if (!(d > 0)) return false;
        const double sii = std::sqrt(d);
        S[(size_t)i * q + i] = sii;
        for (int j = i + 1; j < q; ++j) {
            zc t = G[(size_t)i * q + j];
            for (int k = 0; k < i; ++k) t -= std::conj(S[(size_t)k * q + i]) * S[(size_t)k * q + j];
            S[(size_t)i * q + j] = t / sii;
        }
    }
    return true;
}

// inverse of an upper triangular q x q matrix (row-major)
std::vector<zc> inv_upper(const std::vector<zc>& S, int q) {
    std::vector<zc> X((size_t)q * q, zc(0, 0));
    for (int j = 0; j < q; ++j) {
        X[(size_t)j * q + j] = 1.0 / S[(size_t)j * q + j];
        for (int i = j - 1; i >= 0; --i) {
            zc t = 0;
            for (int k = i + 1; k <= j; ++k) t += S[(size_t)i * q + k] * X[(size_t)k * q + j];
            X[(size_t)i * q + j] = -t / S[(size_t)i * q + i];
        }
    }
    return X;
}

std::vector<zc> mul_upper(const std::vector<zc>& A, const std::vector<zc>& B, int q) {
    std::vector<zc> C((size_t)q * q, zc(0, 0));
    for (int i = 0; i < q; ++i)
        for (int j = i; j < q; ++j) {
            zc t = 0;
            for (int k = i; k <= j; ++k) t += A[(size_t)i * q + k] * B[(size_t)k * q + j];
            C[(size_t)i * q + j] = t;
        }
    return C;
}

// (c, s), c real, with [[c, s], [-conj(s), c]] [a, b]^T = [r, 0]^T
void givens_cs(zc a, zc b, double& c, zc& s) {
    const double aa = std::abs(a), ab = std::abs(b);
    if (ab == 0) {
        c = 1.0;
        s = 0.0;
    } else if (aa == 0) {
        c = 0.0;
        s = std::conj(b) / ab;
    } else {
        const double r = std::hypot(aa, ab);
        c = aa / r;
        s = (a / aa) * std::conj(b) / r;
    }
}

struct Rot {
    int a, b;
    double c;
    zc s;
};
inline void apply_rot(const Rot& R, zc* x) {
    const zc t = R.c * x[R.a] + R.s * x[R.b];
    x[R.b] = -std::conj(R.s) * x[R.a] + R.c * x[R.b];
    x[R.a] = t;
}
}  // namespace

template <typename T>
static hsw_status block_gmres_group(hsw_ctx* ctx, Lane& ln, int prob, const Cx<double>* b,
                                    Cx<double>* x, int64_t ld, int p, const hsw_solve_opts& o,
                                    int* iters_out, double* relres_out) {
    hipStream_t st = ln.st;
    const ProbHost& hp = ctx->ph[prob];
    const ProbDev& Q = ctx->prob_h[prob];
    const int64_t N = hp.Npad;
    const int k = o.restart_k;
    const int LDH = (k + 1) * p;  // rows of the block Hessenberg matrix
    Cx<double> *V = nullptr, *Z = nullptr, *Cd = nullptr, *part = nullptr, *Sd = nullptr;
    double *bn = nullptr, *partn = nullptr;
    int* actd = nullptr;
    {
        const int nchb = bdots_chunks(N), nchn = dots_chunks(N);
        void** slots[] = {(void**)&V, (void**)&Z, (void**)&Cd, (void**)&part, (void**)&Sd,
                          (void**)&bn, (void**)&partn, (void**)&actd};
        const size_t bytes[] = {16 * (size_t)N * LDH, 16 * (size_t)N * k * p, 16 * (size_t)LDH * p,
                                16 * (size_t)nchb * LDH * p, 16 * (size_t)k * p * p, 8 * (size_t)p,
                                8 * (size_t)p * nchn, 4 * (size_t)p};
        const size_t nslot = sizeof(bytes) / sizeof(bytes[0]), base = 16;
        if (ln.gws.size() < base + nslot) ln.gws.resize(base + nslot, {nullptr, 0});
        for (size_t i = 0; i < nslot; ++i) {
            auto& w = ln.gws[base + i];
            if (w.second < bytes[i]) {
                if (w.first) HIPCHK(hipFree(w.first));
                w = {nullptr, 0};
                HIPCHK(hipMalloc(&w.first, bytes[i]));
                w.second = bytes[i];
            }
            *slots[i] = w.first;
        }
    }
    hsw_status s = ensure_solve_ws<T>(ctx, ln, p);
    if (s != HSW_OK) return s;
    std::vector<double> bn_h(p), nrm_h(p), rel(p, 1.0);
    std::vector<int> its(p, 0);
    HIPCHK(hipMemset2DAsync(x, 16 * ld, 0, 16 * N, p, st));
    launch_norm(b, ld, N, p, nullptr, partn, bn, nullptr, 0, st);
    HIPCHK(hipMemcpyAsync(bn_h.data(), bn, 8 * p, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int c = 0; c < p; ++c)
        if (!(bn_h[c] > 0)) rel[c] = 0.0;
    int total = 0;
    std::vector<zc> H, Gr, Cs, Gm;
    // host sources of asynchronous uploads: each is rewritten only after a
    // later synchronisation of the stream, so the upload has completed
    std::vector<zc> Sbuf, Ybuf;
    std::vector<int> actbuf;
    // Cholesky QR of the q vectors at W (in place); false on breakdown.
    auto cholqr = [&](Cx<double>* W, int q, std::vector<zc>& S) -> int {
        std::vector<zc> Sp[2];
        for (int pass = 0; pass < 2; ++pass) {
            launch_bdots(W, N, q, W, N, q, N, part, Cd, st);
            Gm.assign((size_t)q * q, 0);
            if (hipMemcpyAsync(Gm.data(), Cd, 16 * (size_t)q * q, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return -1;
            if (!chol_upper(Gm, q, Sp[pass])) return 0;
            Sbuf = inv_upper(Sp[pass], q);
            if (hipMemcpyAsync(Sd, Sbuf.data(), 16 * (size_t)q * q, hipMemcpyHostToDevice, st) != hipSuccess)
                return -1;
            launch_bcombine(W, N, q, Sd, q, W, N, nullptr, N, 1.0, 0.0, st);
        }
        S = mul_upper(Sp[1], Sp[0], q);
        return 1;
    };
    while (true) {
        // true residual block of every column into V, its norms
        launch_matvec(Q, ctx->d_et, x, V, b, ld, p, 1, st);
        launch_norm(V, N, N, p, nullptr, partn, bn + 0, nullptr, 0, st);
        HIPCHK(hipMemcpyAsync(nrm_h.data(), bn, 8 * p, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::vector<int> act;
        for (int c = 0; c < p; ++c) {
            if (!(bn_h[c] > 0)) continue;
            rel[c] = nrm_h[c] / bn_h[c];
            if (rel[c] >= o.rtol) act.push_back(c);
        }
        if (act.empty() || total >= o.maxit) break;
        const int q = (int)act.size();
        for (int u = 0; u < q; ++u)  // act is increasing: each source lies at or after its target
            if (act[u] != u)
                HIPCHK(hipMemcpyAsync(V + (int64_t)u * N, V + (int64_t)act[u] * N, 16 * (size_t)N,
                                      hipMemcpyDeviceToDevice, st));
        actbuf = act;
        HIPCHK(hipMemcpyAsync(actd, actbuf.data(), 4 * q, hipMemcpyHostToDevice, st));
        std::vector<zc> S0;
        const int ok0 = cholqr(V, q, S0);
        if (ok0 < 0) return fail(ctx, HSW_E_DEVICE, "block GMRES transfer failed");
        if (ok0 == 0) return HSW_E_BREAKDOWN;  // rank-deficient residual block: the caller falls back
        double scale = 0;
        for (int u = 0; u < q; ++u) scale = std::max(scale, std::abs(S0[(size_t)u * q + u]));
        const int ldh = (k + 1) * q;
        H.assign((size_t)ldh * k * q, zc(0, 0));  // column-major, leading dimension ldh
        Gr.assign((size_t)ldh * q, zc(0, 0));     // column c at c * ldh
        for (int c = 0; c < q; ++c)
            for (int r = 0; r <= c; ++r) Gr[(size_t)c * ldh + r] = S0[(size_t)r * q + c];
        std::vector<Rot> rots;
        int jdone = 0;
        for (int j = 0; j < k; ++j) {
            Cx<double>* Vj = V + (int64_t)j * q * N;
            Cx<double>* W = V + (int64_t)(j + 1) * q * N;
            Cx<double>* Zj = Z + (int64_t)j * q * N;
            s = sweep_any<T>(ctx, ln, prob, Vj, Zj, q, N);
            if (s != HSW_OK) return s;
            timed(ctx, "matvec", 1, (double)N * (32.0 * q + 8.0), 56.0 * (double)N * q,
                  [&] { launch_matvec(Q, ctx->d_et, Zj, W, nullptr, N, q, 0, st); });
            total += 1;
            for (int c : act) its[c] += 1;
            const int m = (j + 1) * q;
            Cs.assign((size_t)m * q, zc(0, 0));
            for (int pass = 0; pass < 2; ++pass) {
                launch_bdots(V, N, m, W, N, q, N, part, Cd, st);
                launch_bcombine(V, N, m, Cd, q, W, N, nullptr, N, -1.0, 1.0, st);
                std::vector<zc> Cp((size_t)m * q);
                HIPCHK(hipMemcpyAsync(Cp.data(), Cd, 16 * (size_t)m * q, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                for (size_t e = 0; e < Cp.size(); ++e) Cs[e] += Cp[e];
            }
            std::vector<zc> Sj;
            const int okj = cholqr(W, q, Sj);
            if (okj < 0) return fail(ctx, HSW_E_DEVICE, "block GMRES transfer failed");
            bool breakdown = okj == 0;
            if (!breakdown) {
                double dmin = 1e300, dmax = 0;
                for (int u = 0; u < q; ++u) {
                    const double d = std::abs(Sj[(size_t)u * q + u]);
                    dmin = std::min(dmin, d);
                    dmax = std::max(dmax, d);
                }
                scale = std::max(scale, dmax);
                breakdown = dmin <= 1e-14 * scale;
            }
            // block column j of H: the Gram-Schmidt coefficients over the
            // subdiagonal block Sj (zero on breakdown)
            for (int u = 0; u < q; ++u) {
                zc* col = H.data() + (size_t)(j * q + u) * ldh;
                for (int i = 0; i < m; ++i) col[i] = Cs[(size_t)i * q + u];
                if (!breakdown)
                    for (int v = 0; v <= u; ++v) col[m + v] = Sj[(size_t)v * q + u];
            }
            // the rotations of earlier blocks, then new ones that zero the
            // block's subdiagonal part column by column (each also applied to
            // the block's later columns and to the right-hand side)
            const size_t nold = rots.size();
            for (int u = 0; u < q; ++u)
                for (size_t i = 0; i < nold; ++i) apply_rot(rots[i], H.data() + (size_t)(j * q + u) * ldh);
            for (int u = 0; u < q; ++u) {
                const int t = j * q + u;
                zc* col = H.data() + (size_t)t * ldh;
                for (int r = t + 1; r <= m + u; ++r) {
                    Rot R{t, r, 1.0, 0.0};
                    givens_cs(col[t], col[r], R.c, R.s);
                    for (int u2 = u; u2 < q; ++u2) apply_rot(R, H.data() + (size_t)(j * q + u2) * ldh);
                    for (int c = 0; c < q; ++c) apply_rot(R, Gr.data() + (size_t)c * ldh);
                    col[r] = 0;
                    rots.push_back(R);
                }
            }
            jdone = j + 1;
            bool conv = true;
            for (int u = 0; u < q; ++u) {
                double r2 = 0;
                for (int r = m; r < m + q; ++r) r2 += std::norm(Gr[(size_t)u * ldh + r]);
                if (!(std::sqrt(r2) / bn_h[act[u]] < o.rtol)) conv = false;
            }
            if (conv || breakdown || total >= o.maxit) break;
        }
        // Y = R^{-1} Gr over the first jdone * q rows; x[act] += Z Y
        const int m = jdone * q;
        std::vector<zc>& Y = Ybuf;
        Y.assign((size_t)m * q, zc(0, 0));  // row-major (i, c)
        for (int c = 0; c < q; ++c)
            for (int i = m - 1; i >= 0; --i) {
                zc t = Gr[(size_t)c * ldh + i];
                for (int l = i + 1; l < m; ++l) t -= H[(size_t)l * ldh + i] * Y[(size_t)l * q + c];
                Y[(size_t)i * q + c] = t / H[(size_t)i * ldh + i];
            }
        HIPCHK(hipMemcpyAsync(Cd, Y.data(), 16 * (size_t)m * q, hipMemcpyHostToDevice, st));
        launch_bcombine(Z, N, m, Cd, q, x, ld, actd, N, 1.0, 1.0, st);
        HIPCHK(hipGetLastError());
    }
    bool okc = true;
    for (int c = 0; c < p; ++c) {
        if (iters_out) iters_out[c] = its[c];
        if (relres_out) relres_out[c] = rel[c];
        okc = okc && rel[c] < o.rtol;
    }
    return okc ? HSW_OK : HSW_E_NOCONV;
}

template <typename T>
static hsw_status block_gmres_impl(hsw_ctx* ctx, Lane& ln, int prob, const Cx<double>* b,
                                   Cx<double>* x, int nrhs, const hsw_solve_opts& o, int* iters_out,
                                   double* relres_out) {
    const int64_t ld = ctx->ph[prob].Npad;
    hsw_status worst = HSW_OK;
    for (int g0 = 0; g0 < nrhs; g0 += BLOCK_KRYLOV_MAX) {
        const int ng = std::min(BLOCK_KRYLOV_MAX, nrhs - g0);
        hsw_status s = block_gmres_group<T>(ctx, ln, prob, b + g0 * ld, x + g0 * ld, ld, ng, o,
                                            iters_out + g0, relres_out + g0);
        if (s == HSW_E_BREAKDOWN)  // dependent right-hand sides: one Krylov space per column
            s = gmres_impl<T>(ctx, ln, prob, b + g0 * ld, x + g0 * ld, ng, o, iters_out + g0,
                              relres_out + g0);
        if (s != HSW_OK && s != HSW_E_NOCONV) return s;
        if (s == HSW_E_NOCONV) worst = s;
    }
    return worst;
}

template <typename T>
static hsw_status solve_problem(hsw_ctx* ctx, Lane& ln, int k, const Cx<double>* bk, Cx<double>* xk,
                                int nr, const hsw_solve_opts& o, int* it, double* rr) {
    return ctx->block_gmres ? block_gmres_impl<T>(ctx, ln, k, bk, xk, nr, o, it, rr)
                            : gmres_impl<T>(ctx, ln, k, bk, xk, nr, o, it, rr);
}

// Solve every problem of the context.  With several problems, they are spread
// over up to nlanes lanes (streams with their own workspaces), one host thread
// each, so that the latency-bound launches of small problems overlap; the
// solve-kernel shapes are tuned on lane 0 first.  Work on the lanes is ordered
// after earlier work on the context's stream, and later work after it.
template <typename T>
static hsw_status solve_all(hsw_ctx* ctx, const hsw_c128* const* b, hsw_c128* const* x,
                            const int32_t* nrhs, const hsw_solve_opts& o, std::vector<int>& its,
                            std::vector<double>& rrs, std::vector<int>& offs) {
    const int np = (int)ctx->ph.size();
    const int nl = (ctx->timer.on || np < 2 || ctx->nlanes < 2) ? 1 : std::min(ctx->nlanes, np);
    std::vector<hsw_status> st(np, HSW_OK);
    auto run = [&](int l) {
        for (int k = l; k < np; k += nl)
            st[k] = solve_problem<T>(ctx, ctx->lanes[l], k, (const Cx<double>*)b[k], (Cx<double>*)x[k],
                                     nrhs[k], o, its.data() + offs[k], rrs.data() + offs[k]);
    };
    if (nl == 1) {
        run(0);
    } else {
        // tune the shapes the lanes will use, on lane 0
        // (GMRES sweeps all of a problem's right-hand sides at once; block
        // GMRES sweeps its active columns, any count up to the group size)
        for (int k = 0; k < np; ++k) {
            const int top = ctx->block_gmres ? std::min(nrhs[k], BLOCK_KRYLOV_MAX) : nrhs[k];
            for (int q = ctx->block_gmres ? 1 : top; q <= top; ++q) {
                hsw_status s = ensure_solve_ws<T>(ctx, ctx->lanes[0], q);
                if (s == HSW_OK) s = tune_solve<T>(ctx, q);
                if (s != HSW_OK) return s;
            }
        }
        if ((int)ctx->lanes.size() < nl) ctx->lanes.resize(nl);
        hipEvent_t ev = nullptr;
        HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev, ctx->st));
        for (int l = 1; l < nl; ++l) {
            if (!ctx->lanes[l].st) HIPCHK(hipStreamCreateWithFlags(&ctx->lanes[l].st, hipStreamNonBlocking));
            HIPCHK(hipStreamWaitEvent(ctx->lanes[l].st, ev, 0));
        }
        ctx->in_lanes = true;
        std::vector<std::thread> th;
        for (int l = 1; l < nl; ++l)
            th.emplace_back([&, l] {
                (void)hipSetDevice(ctx->device);
                run(l);
            });
        run(0);
        for (auto& t : th) t.join();
        ctx->in_lanes = false;
        for (int l = 1; l < nl; ++l) {
            HIPCHK(hipEventRecord(ev, ctx->lanes[l].st));
            HIPCHK(hipStreamWaitEvent(ctx->st, ev, 0));
        }
        HIPCHK(hipStreamSynchronize(ctx->st));
        (void)hipEventDestroy(ev);
    }
    hsw_status worst = HSW_OK;
    for (hsw_status s : st) {
        if (s != HSW_OK && s != HSW_E_NOCONV) return s;
        if (s == HSW_E_NOCONV) worst = s;
    }
    return worst;
}

extern "C" hsw_status hsw_solve(hsw_ctx* ctx, const hsw_c128* const* b, hsw_c128* const* x,
                                const int32_t* nrhs, const hsw_solve_opts* opts, hsw_solve_info* info) {
    if (!ctx) return HSW_E_INVAL;
    if (!ctx->factored) return fail(ctx, HSW_E_STATE, "solve before setup");
    if (!b || !x || !nrhs) return fail(ctx, HSW_E_INVAL, "NULL argument");
    hsw_solve_opts o{20, 1000, 1e-5};
    if (opts) o = *opts;
    if (o.restart_k < 1 || o.maxit < 1 || !(o.rtol > 0))
        return fail(ctx, HSW_E_INVAL, "restart_k >= 1, maxit >= 1, rtol > 0 required");
    const int np = (int)ctx->ph.size();
    std::vector<int> offs(np + 1, 0);
    for (int k = 0; k < np; ++k) {
        if (!b[k] || !x[k] || nrhs[k] < 1) return fail(ctx, HSW_E_INVAL, "bad right-hand side block");
        offs[k + 1] = offs[k] + nrhs[k];
    }
    std::vector<int> its(offs[np], 0);
    std::vector<double> rrs(offs[np], 0.0);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, ctx->st));
    const hsw_status worst = ctx->prec == HSW_C128 ? solve_all<double>(ctx, b, x, nrhs, o, its, rrs, offs)
                                                   : solve_all<float>(ctx, b, x, nrhs, o, its, rrs, offs);
    if (worst != HSW_OK && worst != HSW_E_NOCONV) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return worst;
    }
    HIPCHK(hipEventRecord(e1, ctx->st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int itmax = 0;
    for (int r = 0; r < offs[np]; ++r) {
        if (info && info->iters) info->iters[r] = its[r];
        if (info && info->relres) info->relres[r] = rrs[r];
        itmax = std::max(itmax, its[r]);
    }
    if (info) {
        info->iters_max = itmax;
        info->t_setup = ctx->t_setup;
        info->t_solve = ms * 1e-3;
        info->bad_problem = info->bad_panel = info->bad_front = info->bad_pivot = -1;
    }
    if (worst == HSW_E_NOCONV) fail(ctx, HSW_E_NOCONV, "GMRES did not reach rtol within maxit");
    return worst;
}

// ---------------------------------------------------------------------------
extern "C" hsw_status hsw_query(const hsw_ctx* cctx, int32_t prob, const char* key, int64_t* val) {
    hsw_ctx* ctx = const_cast<hsw_ctx*>(cctx);
    if (!ctx || !key || !val) return HSW_E_INVAL;
    if (prob < 0 || prob >= (int)ctx->ph.size()) return fail(ctx, HSW_E_INVAL, "bad problem index");
    const ProbHost& h = ctx->ph[prob];
    std::string k(key);
    auto panel_of = [&](int64_t i) -> const PanelDev* {
        if (i < 0 || i >= h.m) return nullptr;
        return &ctx->pan_h[h.panel_base + i];
    };
    if (k == "N_pad") *val = h.Npad;
    else if (k == "N_int") *val = h.Nint;
    else if (k == "m") *val = h.m;
    else if (k == "N1") *val = h.N[0];
    else if (k == "N2") *val = h.N[1];
    else if (k == "N3") *val = h.N[2];
    else if (k == "levels") *val = h.levels;
    else if (k == "fronts") *val = ctx->classes[ctx->pan_h[h.panel_base].cls].nfront;
    else if (k == "factor_bytes") *val = (int64_t)h.factor_entries * ctx->esz;
    else if (k == "setup_flops") *val = (int64_t)(8.0 * (h.setup_cmac + h.inverse_cmac));
    else if (k == "factor_flops") *val = (int64_t)(8.0 * h.setup_cmac);
    else if (k == "apply_flops") *val = (int64_t)(8.0 * h.apply_cmac);
    else if (k == "panel_lo" || k == "panel_hi" || k == "panel_nz" || k == "panel_artificial" ||
             k == "panel_naux") {
        const PanelDev* P = panel_of(*val);
        if (!P) return fail(ctx, HSW_E_INVAL, "bad panel index");
        if (k == "panel_lo") *val = P->lo;
        else if (k == "panel_hi") *val = P->hi;
        else if (k == "panel_nz") *val = P->nz;
        else if (k == "panel_artificial") *val = P->ga;
        else *val = ctx->classes[P->cls].naux;
    } else {
        return fail(ctx, HSW_E_INVAL, "unknown key " + k);
    }
    return HSW_OK;
}

static const PanelDev* get_panel(hsw_ctx* ctx, int prob, int panel) {
    if (prob < 0 || prob >= (int)ctx->ph.size()) return nullptr;
    const ProbHost& h = ctx->ph[prob];
    if (panel < 0 || panel >= h.m) return nullptr;
    return &ctx->pan_h[h.panel_base + panel];
}

extern "C" hsw_status hsw_get_perm(const hsw_ctx* cctx, int32_t prob, int32_t panel, int32_t* perm_host) {
    hsw_ctx* ctx = const_cast<hsw_ctx*>(cctx);
    if (!ctx || !perm_host) return HSW_E_INVAL;
    const PanelDev* P = get_panel(ctx, prob, panel);
    if (!P) return fail(ctx, HSW_E_INVAL, "bad problem or panel index");
    const PanelClass& c = ctx->classes[P->cls];
    std::memcpy(perm_host, c.perm.data(), 4 * (size_t)c.naux);
    return HSW_OK;
}

extern "C" hsw_status hsw_get_front_info(const hsw_ctx* cctx, int32_t prob, int32_t panel,
                                         int32_t front, int32_t* info, int32_t* urows) {
    hsw_ctx* ctx = const_cast<hsw_ctx*>(cctx);
    if (!ctx || !info) return HSW_E_INVAL;
    const PanelDev* P = get_panel(ctx, prob, panel);
    if (!P) return fail(ctx, HSW_E_INVAL, "bad problem or panel index");
    const PanelClass& c = ctx->classes[P->cls];
    if (front < 0 || front >= c.nfront) return fail(ctx, HSW_E_INVAL, "bad front index");
    info[0] = c.start[front];
    info[1] = c.s[front];
    info[2] = c.u[front];
    info[3] = c.parent[front];
    info[4] = c.depth[front];
    if (urows) std::memcpy(urows, c.ulist.data() + c.uoff[front], 4 * (size_t)c.u[front]);
    return HSW_OK;
}

template <typename T>
static hsw_status copy_block(hsw_ctx* ctx, const void* base, int64_t off, int64_t count,
                             std::vector<Cx<double>>& out) {
    std::vector<Cx<T>> tmp(count);
    HIPCHK(hipMemcpy(tmp.data(), (const Cx<T>*)base + off, sizeof(Cx<T>) * count, hipMemcpyDeviceToHost));
    out.resize(count);
    for (int64_t i = 0; i < count; ++i) out[i] = ccast<double>(tmp[i]);
    return HSW_OK;
}

static hsw_status front_block(hsw_ctx* ctx, int prob, int panel, int front, const void* base,
                              std::vector<Cx<double>>& blk, int& s, int& u) {
    if (!ctx->factored) return fail(ctx, HSW_E_STATE, "factors not available before setup");
    const PanelDev* P = get_panel(ctx, prob, panel);
    if (!P) return fail(ctx, HSW_E_INVAL, "bad problem or panel index");
    if (front < 0 || front >= P->nfront) return fail(ctx, HSW_E_INVAL, "bad front index");
    HIPCHK(hipStreamSynchronize(ctx->st));
    const FrontInst& f = ctx->inst_h[P->inst_base + front];
    s = f.s;
    u = f.u;
    const int64_t cnt = (int64_t)(f.s + f.u) * f.s;
    return ctx->prec == HSW_C128 ? copy_block<double>(ctx, base, f.loff, cnt, blk)
                                 : copy_block<float>(ctx, base, f.loff, cnt, blk);
}

extern "C" hsw_status hsw_get_front(const hsw_ctx* cctx, int32_t prob, int32_t panel, int32_t front,
                                    hsw_c128* D, hsw_c128* L_TL, hsw_c128* F_BL, int32_t* ps,
                                    int32_t* pu) {
    hsw_ctx* ctx = const_cast<hsw_ctx*>(cctx);
    if (!ctx) return HSW_E_INVAL;
    if (!ctx->keep_factors)
        return fail(ctx, HSW_E_STATE,
                    "the factors were overwritten by their selective inverse: set the option "
                    "keep_factors before hsw_setup");
    std::vector<Cx<double>> blk;
    int s = 0, u = 0;
    hsw_status st = front_block(ctx, prob, panel, front, ctx->d_L, blk, s, u);
    if (st != HSW_OK) return st;
    const int n = s + u;
    if (ps) *ps = s;
    if (pu) *pu = u;
    for (int j = 0; j < s; ++j) {
        if (D) D[j] = {blk[(int64_t)j * n + j].re, blk[(int64_t)j * n + j].im};
        if (L_TL)
            for (int i = 0; i < s; ++i) {
                Cx<double> v = i > j ? blk[(int64_t)j * n + i] : cx<double>(i == j ? 1.0 : 0.0, 0.0);
                L_TL[(int64_t)j * s + i] = {v.re, v.im};
            }
        if (F_BL)
            for (int i = 0; i < u; ++i) {
                Cx<double> v = blk[(int64_t)j * n + s + i];
                F_BL[(int64_t)j * u + i] = {v.re, v.im};
            }
    }
    return HSW_OK;
}

extern "C" hsw_status hsw_get_front_inverse(const hsw_ctx* cctx, int32_t prob, int32_t panel,
                                            int32_t front, hsw_c128* G) {
    hsw_ctx* ctx = const_cast<hsw_ctx*>(cctx);
    if (!ctx || !G) return HSW_E_INVAL;
    std::vector<Cx<double>> blk;
    int s = 0, u = 0;
    hsw_status st = front_block(ctx, prob, panel, front, ctx->d_G, blk, s, u);
    if (st != HSW_OK) return st;
    const int g0 = ctx->inst_h[get_panel(ctx, prob, panel)->inst_base + front].g0;
    const int64_t n = (int64_t)s + u;
    for (size_t i = 0; i < blk.size(); ++i)
        G[i] = (int64_t)i < g0 * n ? hsw_c128{0, 0} : hsw_c128{blk[i].re, blk[i].im};
    return HSW_OK;
}

extern "C" hsw_status hsw_kernel_timing(hsw_ctx* ctx, const char* kernel, int32_t enable,
                                        int64_t* launches, double* seconds, double* bytes,
                                        double* flops) {
    if (!ctx || !kernel) return HSW_E_INVAL;
    static const char* known[] = {"fwd", "bwd", "scatter", "diag", "panel", "trailing", "schur",
                                  "assemble", "inverse", "matvec"};
    bool ok = false;
    for (const char* k : known) ok = ok || std::strcmp(k, kernel) == 0;
    if (!ok) return fail(ctx, HSW_E_INVAL, std::string("unknown kernel class ") + kernel);
    KernelTimer& t = ctx->timer;
    auto drop = [&]() {
        for (auto& e : t.ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        t.ev.clear();
    };
    if (enable) {
        HIPCHK(hipStreamSynchronize(ctx->st));
        drop();
        t.kernel = kernel;
        t.on = true;
        t.launches = 0;
        t.bytes = t.flops = 0;
        return HSW_OK;
    }
    HIPCHK(hipStreamSynchronize(ctx->st));
    double sec = 0;
    for (auto& e : t.ev) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e.first, e.second));
        sec += ms * 1e-3;
    }
    if (launches) *launches = t.launches;
    if (seconds) *seconds = sec;
    if (bytes) *bytes = t.bytes;
    if (flops) *flops = t.flops;
    drop();
    t.on = false;
    return HSW_OK;
}
