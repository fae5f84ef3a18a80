/*
 * Host runtime behind the C ABI declared in include/ad.h: parameter
 * validation, the work list of the pair kernel, the workspace layout, the
 * step loop (direct launches or a captured HIP graph) and error reporting.
 */
#include <hip/hip_runtime.h>
#include <math.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/ad.h"
#include "ad_internal.h"
#include "ad_order.h"

using ad::Coef;
using ad::Ctl;
using ad::Dev;
using ad::Item;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kTabSteps = 4096;          /* steps per table chunk */
/* steps per graph of a run of steps, longest first: a run replays the
 * longest graph that fits before the next record point or table chunk */
constexpr int kGraphSteps[] = {16, 4, 1};
constexpr int kGraphs = 3;
constexpr int kRing = 2 * kTabSteps;     /* table entries (two chunks) */
static_assert((kRing & (kRing - 1)) == 0, "the kernels take table rows as step & (ring - 1)");

/* message of the last failure of a context-free call on this thread
 * (ad_create, ad_mobility_apply_static); a fixed buffer, so that setting it
 * allocates nothing */
thread_local char g_thread_error[512];

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

struct ad_ctx {
    ad_params p{};
    Coef coef{};
    double omega = 0.0;
    int nsys = 0;
    std::vector<int32_t> S;
    std::vector<int32_t> off; /* sphere offsets, nsys+1 */
    std::vector<int32_t> dsys;
    int Ntot = 0, Stot = 0;
    ad_launch launch{};
    std::vector<Item> items;
    std::vector<int32_t> sysP;
    std::vector<long long> pbase;
    long long npart = 0;
    std::vector<long long> hbase; /* dense mode: first tensor element per system */
    std::vector<Item> fitems;     /* fused stages of an ensemble: (system, target block) */
    bool fused_ready = false;     /* the fused kernels may use all of LDS */
    long long nH = 0;             /* dense mode: tensor elements over all systems */
    int maxNb = 0;

    /* workspace */
    void* ws = nullptr;
    uint64_t ws_bytes = 0;
    Dev dev{};     /* even stages: read pack 0, write pack 1 */
    Dev dev_odd{}; /* odd stages: read pack 1, write pack 0 */
    bool state = false;
    /* the first pack holds the state's stage-0 pack (written by the last
     * stage of the previous step call); anything that overwrites or moves it
     * clears this */
    bool pack_valid = false;
    /* the device step slot holds c->step (every staged step leaves it so) */
    bool slot_valid = false;
    /* steps [tab_lo, tab_hi) have their rows in the device step table */
    long long tab_lo = 0, tab_hi = 0;
    double t0 = 0.0;
    long long step = 0;

    /* pinned host staging */
    double* h_tab = nullptr;    /* kRing*8 */
    double2* h_phi = nullptr;   /* Stot (sin phi, cos phi) */
    double* h_phi_in = nullptr; /* Stot phases copied from the caller's device array */
    int* h_flag = nullptr;
    hipEvent_t tab_event = nullptr;
    bool tab_event_live = false;

    /* graphs of kGraphSteps[g] steps: one graph launch costs several
     * microseconds, so runs of steps replay the longest graph that fits */
    bool use_graph = false;
    hipGraphExec_t graph_exec[kGraphs] = {};
    hipGraph_t graph[kGraphs] = {};
    hipStream_t capture_stream = nullptr;

    /* pair-kernel timing */
    bool profile = false;
    std::vector<hipEvent_t> ev;  /* start/stop pairs */
    int ev_used = 0;
    double prof_ms = 0.0;
    long long prof_launches = 0;

    std::string err;
};

static int fail(ad_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        memcpy(g_thread_error, buf, sizeof g_thread_error);
    return code;
}

namespace ad {
int thread_fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_thread_error, sizeof g_thread_error, fmt, ap);
    va_end(ap);
    return code;
}
void thread_clear_error() { g_thread_error[0] = 0; }

Coef make_coef(const ad_params* p) {
    Coef k{};
    k.cs = 1.0 / (6.0 * kPi * p->eta * p->a);
    k.co = 1.0 / (8.0 * kPi * p->eta);
    k.k = p->k;
    k.ell = p->ell;
    k.lam = p->lambda;
    k.dt = p->dt;
    k.h2 = 0.5 * p->dt;
    k.dt6 = p->dt / 6.0;
    k.ks = p->steric_k;
    k.rc = p->steric_r;
    k.cr = 2.0 * p->a * p->a / (24.0 * kPi * p->eta);
    k.crr = (float)(2.0 * p->a * p->a / 3.0);
    k.crr64 = 2.0 * p->a * p->a / 3.0;
    k.rpy = p->tensor == AD_RPY ? 1 : 0;
    k.noise = p->kT > 0.0 ? 1 : 0;
    k.g = sqrt(2.0 * p->kT * (1.0 / (6.0 * kPi * p->eta * p->a)) * p->dt);
    k.seed = p->seed;
    return k;
}
}  // namespace ad

#define HIPCHECK(ctx, expr)                                                                       \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, AD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

/* ------------------------------------------------------------ work list */

static bool is_dense(const ad_ctx* c) { return c->p.precision == AD_FP64_DENSE; }
static int prec_of(const ad_ctx* c);

/* dense mode: tensor bytes over all systems, 72 Nb^2 each */
static double dense_bytes(int nsys, const int32_t* S) {
    double b = 0.0;
    for (int q = 0; q < nsys; ++q) b += 72.0 * (2.0 * S[q]) * (2.0 * S[q]);
    return b;
}
constexpr double kDenseMaxBytes = 34359738368.0; /* 32 GiB */

static ad_launch default_launch(const ad_ctx* c) {
    ad_launch L{};
    int maxN = 0;
    for (int b = 0; b < c->nsys; ++b) maxN = std::max(maxN, 2 * c->S[b]);
    L.wj = 1;
    L.posmode = c->p.precision == AD_FP32C ? AD_POS_HILO : 0;
    if (is_dense(c)) {
        /* about 2048 product items: row blocks x j-chunks */
        L.wg = ad::DENSE_ROWS;
        L.ipl = 1;
        const int rb = (3 * maxN + ad::DENSE_ROWS - 1) / ad::DENSE_ROWS;
        const int P = std::max(1, 2048 / rb);
        int jc = (maxN + P - 1) / P;
        jc = std::min(ad::DENSE_JMAX, std::max(64, (jc + 63) / 64 * 64));
        L.jchunk = jc;
        return L;
    }
    const ad::PairShape sh = ad::default_pair_shape(prec_of(c), c->nsys, maxN);
    L.ipl = sh.ipl;
    L.wg = sh.wg;
    L.wj = sh.wj;
    L.jchunk = sh.jchunk;
    return L;
}

static int validate_launch(ad_ctx* c, const ad_launch& L) {
    if (is_dense(c)) {
        if (L.wg != ad::DENSE_ROWS || L.ipl != 1 || L.wj != 1 || L.posmode != 0 || L.fused != 0)
            return fail(c, AD_EINVAL, "AD_FP64_DENSE takes wg %d, ipl 1, wj 1, posmode 0", ad::DENSE_ROWS);
        if (L.jchunk < 64 || L.jchunk > ad::DENSE_JMAX)
            return fail(c, AD_EINVAL, "AD_FP64_DENSE: launch.jchunk must be in [64, %d]", ad::DENSE_JMAX);
        return AD_OK;
    }
    if (L.wg != 64 && L.wg != 256) return fail(c, AD_EINVAL, "launch.wg must be 64 or 256 (got %d)", L.wg);
    if (L.ipl != 1 && L.ipl != 2 && L.ipl != 4) return fail(c, AD_EINVAL, "launch.ipl must be 1, 2 or 4");
    if (L.wj != 1 && !(L.wj == 4 && L.wg == 256 && c->p.precision == AD_FP32C))
        return fail(c, AD_EINVAL, "launch.wj must be 1, or 4 with wg 256 in AD_FP32C");
    if (c->p.precision != AD_FP32C && L.ipl > 2) return fail(c, AD_EINVAL, "FP64 modes support ipl 1 or 2");
    if (c->p.precision == AD_FP32C && L.posmode != AD_POS_HILO && L.posmode != AD_POS_SINGLE)
        return fail(c, AD_EINVAL, "launch.posmode must be AD_POS_HILO or AD_POS_SINGLE");
    if (L.jchunk < 64 && c->p.precision != AD_FP64) return fail(c, AD_EINVAL, "launch.jchunk must be >= 64");
    if (L.fused < 0 || L.fused > 4) return fail(c, AD_EINVAL, "launch.fused must be 0, 1, 2, 3 or 4");
    if (L.fused == 4) {
        const int p64 = c->p.precision != AD_FP32C;
        if (c->p.steric_k != 0.0) return fail(c, AD_EINVAL, "launch.fused 4 takes no steric forces");
        const int lim = p64 ? ad::RES_MAX64 : ad::RES_MAX32;
        if (c->maxNb > lim)
            return fail(c, AD_EINVAL, "launch.fused 4: systems of at most %d spheres in this precision (got %d)", lim,
                        c->maxNb);
        return AD_OK;
    }
    if (L.fused == 3 && c->p.precision == AD_FP64_TILED) {
        /* the FP64 streamed stage: every system size, no steric forces */
        if (c->p.steric_k != 0.0) return fail(c, AD_EINVAL, "launch.fused 3 takes no steric forces");
        if (ad::fused_stream64_lds_bytes() > ad::FUSED_LDS_MAX) return fail(c, AD_EINVAL, "launch.fused 3: LDS");
        return AD_OK;
    }
    if (L.fused) {
        if (c->p.precision != AD_FP32C || c->p.steric_k != 0.0)
            return fail(c, AD_EINVAL, "launch.fused 1 and 2 need AD_FP32C (3 also AD_FP64_TILED) and no steric "
                        "forces");
        const int hilo = L.posmode == AD_POS_HILO;
        const int lds = L.fused == 3   ? ad::fused_stream_lds_bytes(hilo)
                        : L.fused == 2 ? ad::fused_wide_lds_bytes(c->maxNb, hilo)
                                       : ad::fused_lds_bytes(c->maxNb, hilo, c->nsys > 1 ? 4 : 16);
        if (lds > ad::FUSED_LDS_MAX)
            return fail(c, AD_EINVAL, "launch.fused: a system of %d spheres does not fit in LDS with this "
                        "position mode", c->maxNb);
    }
    return AD_OK;
}

/* FP32C with steric forces: the pair kernel records steric candidates */
static bool uses_lists(const ad_ctx* c) { return c->p.steric_k != 0.0 && c->p.precision == AD_FP32C; }

static ad::Shape shape_of(const ad_ctx* c) {
    ad::Shape sh;
    sh.wg = c->launch.wg;
    sh.wj = c->launch.wj;
    sh.ipl = c->launch.ipl;
    sh.split = c->launch.posmode == AD_POS_HILO ? 1 : 0;
    sh.fused = c->launch.fused;
    sh.steric = uses_lists(c) ? 1 : 0;
    sh.rpy = c->p.tensor == AD_RPY ? 1 : 0;
    return sh;
}

/* partial-sum components per sphere: FP64 with RPY keeps the correction apart */
static int ncomp_of(const ad_ctx* c) {
    return (c->p.tensor == AD_RPY && (c->p.precision == AD_FP64 || c->p.precision == AD_FP64_TILED)) ? 6 : 3;
}

/* dense mode: product items of DENSE_ROWS tensor rows x jchunk source
 * spheres; i0 and ni count local tensor rows */
static void build_dense_items(ad_ctx* c) {
    const int jc0 = c->launch.jchunk;
    c->items.clear();
    c->sysP.assign(c->nsys, 1);
    c->pbase.assign(c->nsys, 0);
    c->hbase.assign(c->nsys, 0);
    long long pb = 0, hb = 0;
    for (int b = 0; b < c->nsys; ++b) {
        const int Nb = 2 * c->S[b];
        const int jc = std::min(jc0, Nb);
        const int P = (Nb + jc - 1) / jc;
        c->sysP[b] = P;
        c->pbase[b] = pb;
        c->hbase[b] = hb;
        pb += (long long)P * 3 * Nb;
        hb += 9LL * Nb * Nb;
        for (int ch = 0; ch < P; ++ch)
            for (int r = 0; r < 3 * Nb; r += ad::DENSE_ROWS) {
                Item it;
                it.sys = b;
                it.i0 = r;
                it.ni = std::min(ad::DENSE_ROWS, 3 * Nb - r);
                it.j0 = c->off[b] + ch * jc;
                it.nj = std::min(jc, Nb - ch * jc);
                it.c = ch;
                it.Nb = Nb;
                it.ioff = c->off[b];
                c->items.push_back(it);
            }
    }
    c->npart = pb;
    c->nH = hb;
    std::stable_sort(c->items.begin(), c->items.end(), [](const Item& a, const Item& b) {
        return (long long)a.ni * a.nj > (long long)b.ni * b.nj;
    });
}

static void build_items(ad_ctx* c) {
    const ad_launch& L = c->launch;
    const int NC = ncomp_of(c);
    if (is_dense(c)) {
        build_dense_items(c);
        return;
    }
    c->items.clear();
    c->sysP.assign(c->nsys, 1);
    c->pbase.assign(c->nsys, 0);
    c->hbase.assign(c->nsys, 0);
    c->nH = 0;
    long long pb = 0;
    const int IB = L.ipl * L.wg / L.wj;
    for (int b = 0; b < c->nsys; ++b) {
        const int Nb = 2 * c->S[b];
        const int jc = (c->p.precision == AD_FP64) ? Nb : std::min(L.jchunk, Nb);
        const int P = (Nb + jc - 1) / jc;
        c->sysP[b] = P;
        c->pbase[b] = pb;
        pb += (long long)P * NC * Nb;
        for (int ch = 0; ch < P; ++ch) {
            const int j0 = c->off[b] + ch * jc;
            const int nj = std::min(jc, Nb - ch * jc);
            for (int i = 0; i < Nb; i += IB) {
                Item it;
                it.sys = b;
                it.i0 = c->off[b] + i;
                it.ni = std::min(IB, Nb - i);
                it.j0 = j0;
                it.nj = nj;
                it.c = ch;
                it.Nb = Nb;
                it.ioff = c->off[b];
                c->items.push_back(it);
            }
        }
    }
    c->npart = pb;
    /* AD_FP64 with two kernels per stage: the pair sum's work list, blocks of
     * TW targets (one work-group each), longest system first (ad_kernels.hip,
     * k_pairs_f64w) */
    c->fitems.clear();
    if (c->p.precision == AD_FP64 && L.fused == 0) {
        const int tb = ad::f64w_targets(c->Ntot);
        for (int b = 0; b < c->nsys; ++b) {
            const int Nb = 2 * c->S[b];
            for (int i = 0; i < Nb; i += tb) {
                Item it{};
                it.sys = b;
                it.i0 = c->off[b] + i;
                it.ni = std::min(tb, Nb - i);
                it.j0 = c->off[b];
                it.nj = Nb;
                it.ioff = c->off[b];
                it.Nb = Nb;
                c->fitems.push_back(it);
            }
        }
        std::stable_sort(c->fitems.begin(), c->fitems.end(), [](const Item& x, const Item& y) { return x.Nb > y.Nb; });
    }
    /* fused stages: one item per target block of a system (16 targets for an
     * ensemble in the first and the streamed form, 64 in the wide form, for
     * one system too), longest system first */
    if (c->launch.fused == 4) {
        /* resident form: one work-group per system, longest first */
        for (int b = 0; b < c->nsys; ++b) {
            Item it{};
            it.sys = b;
            it.i0 = c->off[b];
            it.ni = 2 * c->S[b];
            it.ioff = c->off[b];
            it.Nb = 2 * c->S[b];
            c->fitems.push_back(it);
        }
        std::stable_sort(c->fitems.begin(), c->fitems.end(),
                         [](const Item& a, const Item& b) { return a.Nb > b.Nb; });
    } else if (((c->launch.fused == 1 || c->launch.fused == 3) && c->nsys > 1) || c->launch.fused == 2) {
        const int blk = c->launch.fused == 2 ? ad::FW_I : c->launch.fused == 3 ? ad::stream_targets(c->Ntot) : 16;
        for (int b = 0; b < c->nsys; ++b) {
            const int Nb = 2 * c->S[b];
            for (int i = 0; i < Nb; i += blk) {
                Item it{};
                it.sys = b;
                it.i0 = c->off[b] + i;
                it.ni = std::min(blk, Nb - i);
                it.ioff = c->off[b];
                it.Nb = Nb;
                c->fitems.push_back(it);
            }
        }
        std::stable_sort(c->fitems.begin(), c->fitems.end(),
                         [](const Item& a, const Item& b) { return a.Nb > b.Nb; });
        ad::xcd_order(c->fitems);
    }
    /* longest first: the hardware dispatcher then hands the cheap items to
     * whichever compute units free up last */
    std::stable_sort(c->items.begin(), c->items.end(), [](const Item& a, const Item& b) {
        return (long long)a.ni * a.nj > (long long)b.ni * b.nj;
    });
}

/* ------------------------------------------------------------ workspace */

struct Layout {
    size_t ctl, X, R, U0, Y, Fs, nbr_cnt, nbr_idx, phitrig, dsys, sys_off, sys_P, sys_pbase, sys_hbase, items,
        pA, pB, pC, pD, pA2, pB2, pC2, pD2, part, tab, H, fitems, total;
};

static Layout layout(const ad_ctx* c) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t N = c->Ntot, S = c->Stot;
    L.ctl = take(sizeof(Ctl));
    L.X = take(3 * N * 8);
    L.R = take(3 * N * 8);
    L.U0 = take(3 * N * 8);
    const bool steric = c->p.steric_k != 0.0;
    L.Y = take(steric ? 3 * N * 8 : 0);
    L.Fs = take(steric ? 3 * N * 8 : 0);
    L.nbr_cnt = take(uses_lists(c) ? N * 4 : 0);
    L.nbr_idx = take(uses_lists(c) ? N * 4 * ad::NBR_CAP : 0);
    L.phitrig = take(S * 16);
    L.dsys = take(S * 4);
    L.sys_off = take((c->nsys + 1) * 4);
    L.sys_P = take(c->nsys * 4);
    L.sys_pbase = take(c->nsys * 8);
    L.sys_hbase = take(c->nsys * 8);
    L.items = take(std::max<size_t>(1, c->items.size()) * sizeof(Item));
    const bool f32 = c->p.precision == AD_FP32C;
    L.pA = take(f32 ? N * 16 : 0);
    L.pB = take(f32 ? N * 16 : 0);
    L.pC = take(f32 ? N * 8 : 0);
    L.pD = take(f32 ? 0 : 3 * N * 16);
    L.pA2 = take(f32 ? N * 16 : 0);
    L.pB2 = take(f32 ? N * 16 : 0);
    L.pC2 = take(f32 ? N * 8 : 0);
    L.pD2 = take(f32 ? 0 : 3 * N * 16);
    L.part = take((size_t)c->npart * 8);
    L.tab = take((size_t)kRing * 8 * 8);
    L.H = take((size_t)c->nH * 8);
    L.fitems = take(c->fitems.size() * sizeof(Item));
    L.total = o;
    return L;
}

static void make_dev(ad_ctx* c) {
    /* the step table and the control block are re-laid out: nothing in them
     * is current any more */
    c->tab_lo = c->tab_hi = 0;
    c->slot_valid = false;
    Layout L = layout(c);
    char* b = static_cast<char*>(c->ws);
    Dev& d = c->dev;
    d.ctl = reinterpret_cast<Ctl*>(b + L.ctl);
    d.X = reinterpret_cast<double*>(b + L.X);
    d.R = reinterpret_cast<double*>(b + L.R);
    d.U0 = reinterpret_cast<double*>(b + L.U0);
    d.Y = reinterpret_cast<double*>(b + L.Y);
    d.Fs = reinterpret_cast<double*>(b + L.Fs);
    d.nbr_cnt = uses_lists(c) ? reinterpret_cast<int*>(b + L.nbr_cnt) : nullptr;
    d.nbr_idx = uses_lists(c) ? reinterpret_cast<int*>(b + L.nbr_idx) : nullptr;
    {
        /* skin of half the contact distance: listed below 1.5 rc, valid while
         * no sphere moves more than rc/4 between stages */
        const double skin = 0.5 * c->p.steric_r;
        d.list_r2 = (float)((c->p.steric_r + skin) * (c->p.steric_r + skin));
        d.move2 = 0.25 * skin * skin;
    }
    d.phitrig = reinterpret_cast<const double2*>(b + L.phitrig);
    d.dsys = reinterpret_cast<const int*>(b + L.dsys);
    d.sys_off = reinterpret_cast<const int*>(b + L.sys_off);
    d.sys_P = reinterpret_cast<const int*>(b + L.sys_P);
    d.sys_pbase = reinterpret_cast<const long long*>(b + L.sys_pbase);
    d.sys_hbase = reinterpret_cast<const long long*>(b + L.sys_hbase);
    d.H = c->nH ? reinterpret_cast<double*>(b + L.H) : nullptr;
    d.fitems = reinterpret_cast<const Item*>(b + L.fitems);
    d.nfitems = (int)c->fitems.size();
    d.items = reinterpret_cast<const Item*>(b + L.items);
    d.pA = reinterpret_cast<float4*>(b + L.pA);
    d.pB = reinterpret_cast<float4*>(b + L.pB);
    d.pC = reinterpret_cast<float2*>(b + L.pC);
    d.pD = reinterpret_cast<double2*>(b + L.pD);
    d.pA2 = reinterpret_cast<float4*>(b + L.pA2);
    d.pB2 = reinterpret_cast<float4*>(b + L.pB2);
    d.pC2 = reinterpret_cast<float2*>(b + L.pC2);
    d.pD2 = reinterpret_cast<double2*>(b + L.pD2);
    d.part = reinterpret_cast<double*>(b + L.part);
    d.tab = reinterpret_cast<const double*>(b + L.tab);
    d.ring = kRing;
    d.Ntot = c->Ntot;
    d.Stot = c->Stot;
    d.nsys = c->nsys;
    d.nitems = (int)c->items.size();
    d.ncomp = ncomp_of(c);
    Dev& o = c->dev_odd;
    o = d;
    o.pA = d.pA2;
    o.pB = d.pB2;
    o.pC = d.pC2;
    o.pD = d.pD2;
    o.pA2 = d.pA;
    o.pB2 = d.pB;
    o.pC2 = d.pC;
    o.pD2 = d.pD;
}

static void drop_graph(ad_ctx* c) {
    for (int g = 0; g < kGraphs; ++g) {
        if (c->graph_exec[g]) (void)hipGraphExecDestroy(c->graph_exec[g]);
        if (c->graph[g]) (void)hipGraphDestroy(c->graph[g]);
        c->graph_exec[g] = nullptr;
        c->graph[g] = nullptr;
    }
}

/* upload the work list and the per-system tables (synchronous) */
static int upload_tables(ad_ctx* c) {
    Layout L = layout(c);
    char* b = static_cast<char*>(c->ws);
    HIPCHECK(c, hipMemcpy(b + L.dsys, c->dsys.data(), c->Stot * 4, hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(b + L.sys_off, c->off.data(), (c->nsys + 1) * 4, hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(b + L.sys_P, c->sysP.data(), c->nsys * 4, hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(b + L.sys_pbase, c->pbase.data(), c->nsys * 8, hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(b + L.sys_hbase, c->hbase.data(), c->nsys * 8, hipMemcpyHostToDevice));
    if (!c->items.empty())
        HIPCHECK(c, hipMemcpy(b + L.items, c->items.data(), c->items.size() * sizeof(Item), hipMemcpyHostToDevice));
    if (!c->fitems.empty())
        HIPCHECK(c, hipMemcpy(b + L.fitems, c->fitems.data(), c->fitems.size() * sizeof(Item),
                              hipMemcpyHostToDevice));
    return AD_OK;
}

/* ------------------------------------------------------------ step pieces */

static int prec_of(const ad_ctx* c) {
    return c->p.precision == AD_FP32C ? ad::PREC_FP32C
                                      : (c->p.precision == AD_FP64_TILED ? ad::PREC_FP64_TILED : ad::PREC_FP64);
}

/* (sin, cos) of omega*t on the host (libm) */
static void trig_at(const ad_ctx* c, double t, double* s, double* co) {
    double wt = c->omega * t;
    *s = sin(wt);
    *co = cos(wt);
}

/* Make the device table hold steps [s0, s0 + count), count <= kTabSteps:
 * nothing to do if they are there; else the rows of kTabSteps steps from s0
 * are computed and copied, so that runs of a few steps at a time copy once
 * per kTabSteps steps. */
static int fill_table(ad_ctx* c, long long s0, int count, hipStream_t st) {
    if (s0 >= c->tab_lo && s0 + count <= c->tab_hi) return AD_OK;
    count = kTabSteps;
    if (c->tab_event_live) HIPCHECK(c, hipEventSynchronize(c->tab_event));
    const double dt = c->p.dt;
    for (int q = 0; q < count; ++q) {
        const long long n = s0 + q;
        const long long e = n % kRing;
        double* row = c->h_tab + e * 8;
        const double tn = c->t0 + (double)n * dt;
        const double tnext = c->t0 + (double)(n + 1) * dt;
        if (c->p.integrator == AD_RK4) {
            const double th = tn + 0.5 * dt, te = tn + dt;
            trig_at(c, th, &row[0], &row[1]);
            trig_at(c, th, &row[2], &row[3]);
            trig_at(c, te, &row[4], &row[5]);
            trig_at(c, tnext, &row[6], &row[7]);
        } else {
            const double te = tn + dt;
            trig_at(c, te, &row[0], &row[1]);
            trig_at(c, tnext, &row[2], &row[3]);
            row[4] = row[5] = row[6] = row[7] = 0.0;
        }
    }
    const long long e0 = s0 % kRing;
    const long long first = std::min<long long>(count, kRing - e0);
    double* dtab = const_cast<double*>(c->dev.tab);
    HIPCHECK(c, hipMemcpyAsync(dtab + e0 * 8, c->h_tab + e0 * 8, first * 8 * sizeof(double),
                               hipMemcpyHostToDevice, st));
    if (first < count)
        HIPCHECK(c, hipMemcpyAsync(dtab, c->h_tab, (count - first) * 8 * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHECK(c, hipEventRecord(c->tab_event, st));
    c->tab_event_live = true;
    c->tab_lo = s0;
    c->tab_hi = s0 + count;
    return AD_OK;
}

constexpr int kEventPairs = 512;

/* sum the recorded pair-kernel intervals and recycle the events */
static int profile_flush(ad_ctx* c) {
    for (int q = 0; q < c->ev_used; ++q) {
        float ms = 0.f;
        HIPCHECK(c, hipEventSynchronize(c->ev[2 * q + 1]));
        HIPCHECK(c, hipEventElapsedTime(&ms, c->ev[2 * q], c->ev[2 * q + 1]));
        c->prof_ms += ms;
        c->prof_launches += 1;
    }
    c->ev_used = 0;
    return AD_OK;
}

static ad::Epi epi_of(const ad_ctx* c, int stage, double* u_aos) {
    ad::Epi e;
    e.c = c->coef;
    e.prec = prec_of(c);
    e.integ = c->p.integrator;
    e.stage = stage;
    e.nst = c->p.integrator == AD_RK4 ? 4 : 2;
    e.pack_next = c->p.steric_k == 0.0 ? 1 : 0;
    e.u_aos = u_aos;
    return e;
}

static int launch_pairs_timed(ad_ctx* c, const Dev& d, const ad::Epi& e, int mode, hipStream_t st) {
    const ad::Shape sh = shape_of(c);
    const bool fused = mode == 1 && c->launch.fused;
    if (!c->profile) {
        if (fused) {
            HIPCHECK(c, ad::launch_fused(d, e, sh, c->maxNb, st));
            return AD_OK;
        }
        if (is_dense(c))
            HIPCHECK(c, ad::launch_dense(d, e, mode, c->maxNb, st));
        else
            HIPCHECK(c, ad::launch_pairs(d, e, sh, mode, st));
        return AD_OK;
    }
    if (c->ev.empty()) {
        c->ev.resize(2 * kEventPairs);
        for (auto& ev : c->ev) HIPCHECK(c, hipEventCreate(&ev));
    }
    if (c->ev_used == kEventPairs) {
        int rc = profile_flush(c);
        if (rc != AD_OK) return rc;
    }
    if (fused)
        HIPCHECK(c, ad::launch_fused(d, e, sh, c->maxNb, st, c->ev[2 * c->ev_used], c->ev[2 * c->ev_used + 1]));
    else if (is_dense(c))
        HIPCHECK(c, ad::launch_dense(d, e, mode, c->maxNb, st, c->ev[2 * c->ev_used], c->ev[2 * c->ev_used + 1]));
    else
        HIPCHECK(c, ad::launch_pairs(d, e, sh, mode, st, c->ev[2 * c->ev_used], c->ev[2 * c->ev_used + 1]));
    c->ev_used += 1;
    return AD_OK;
}

/* a run of nsteps steps in the resident form, timed like a pair launch */
static int launch_resident_timed(ad_ctx* c, long long step0, int nsteps, double st0, double ct0, hipStream_t st) {
    const ad::Epi e = epi_of(c, 0, nullptr);
    const int hilo = c->launch.posmode == AD_POS_HILO ? 1 : 0;
    if (!c->profile) {
        HIPCHECK(c, ad::launch_resident(c->dev, e, hilo, c->maxNb, step0, nsteps, st0, ct0, st));
        return AD_OK;
    }
    if (c->ev.empty()) {
        c->ev.resize(2 * kEventPairs);
        for (auto& ev : c->ev) HIPCHECK(c, hipEventCreate(&ev));
    }
    if (c->ev_used == kEventPairs) {
        int rc = profile_flush(c);
        if (rc != AD_OK) return rc;
    }
    HIPCHECK(c, ad::launch_resident(c->dev, e, hilo, c->maxNb, step0, nsteps, st0, ct0, st, c->ev[2 * c->ev_used],
                                    c->ev[2 * c->ev_used + 1]));
    c->ev_used += 1;
    return AD_OK;
}

/* launches of one step (no table, no initial pack) */
static int launch_step_kernels(ad_ctx* c, hipStream_t st) {
    const int nst = c->p.integrator == AD_RK4 ? 4 : 2;
    const bool steric = c->p.steric_k != 0.0;
    for (int s = 0; s < nst; ++s) {
        const Dev& d = (s & 1) ? c->dev_odd : c->dev;
        const ad::Epi e = epi_of(c, s, nullptr);
        int rc = launch_pairs_timed(c, d, e, 1, st);
        if (rc != AD_OK) return rc;
        if (c->launch.fused) continue; /* the fused kernel did the epilogue */
        HIPCHECK(c, ad::launch_epilogue(d, e, st));
        if (steric) HIPCHECK(c, ad::launch_steric_pack(d, c->coef, e.prec, st));
    }
    return AD_OK;
}

/* capture nsteps consecutive steps into *graph / *exec */
static int capture_steps(ad_ctx* c, int nsteps, hipGraph_t* graph, hipGraphExec_t* exec) {
    HIPCHECK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = AD_OK;
    for (int k = 0; k < nsteps && rc == AD_OK; ++k) rc = launch_step_kernels(c, c->capture_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
    if (rc != AD_OK) {
        if (g) (void)hipGraphDestroy(g); /* the launch error is the one reported */
        return rc;
    }
    if (e != hipSuccess) return fail(c, AD_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    *graph = g;
    HIPCHECK(c, hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
    return AD_OK;
}

/* capture every graph and upload each to the device on the call's stream,
 * so that the first replay of each pays no upload */
static int ensure_graph(ad_ctx* c, hipStream_t st) {
    if (c->graph_exec[kGraphs - 1]) return AD_OK;
    drop_graph(c);
    if (!c->capture_stream) HIPCHECK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    int rc = AD_OK;
    for (int g = 0; g < kGraphs && rc == AD_OK; ++g) {
        rc = capture_steps(c, kGraphSteps[g], &c->graph[g], &c->graph_exec[g]);
        if (rc == AD_OK && hipGraphUpload(c->graph_exec[g], st) != hipSuccess)
            rc = fail(c, AD_EDEVICE, "hipGraphUpload failed");
    }
    if (rc != AD_OK) drop_graph(c);
    return rc;
}

static int advance(ad_ctx* c, long long nsteps, int record_every, double* centres, double* com, hipStream_t st) {
    if (!c->ws) return fail(c, AD_ESTATE, "no workspace bound");
    if (!c->state) return fail(c, AD_ESTATE, "no state loaded (ad_set_state)");
    if (c->launch.fused && !c->fused_ready) {
        /* before any launch or capture of the step */
        HIPCHECK(c, ad::prepare_fused());
        c->fused_ready = true;
    }
    if (nsteps < 0) return fail(c, AD_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return AD_OK;
    const int prec = prec_of(c);
    const bool resident = c->launch.fused == 4;
    const bool graph = c->use_graph && !c->profile && !resident;
    if (graph) {
        int rc = ensure_graph(c, st);
        if (rc != AD_OK) return rc;
    }
    if (!c->slot_valid) HIPCHECK(c, ad::launch_set_step(c->dev, c->step, st));
    c->slot_valid = false; /* until this call completes */
    if (!c->pack_valid && !resident) {
        double s0, c0;
        trig_at(c, c->t0 + (double)c->step * c->p.dt, &s0, &c0);
        HIPCHECK(c, ad::launch_pack_state(c->dev, c->coef, prec, s0, c0, st));
    }
    c->pack_valid = false; /* until this call completes */
    long long done = 0, rec = 0;
    while (done < nsteps) {
        const int chunk = (int)std::min<long long>(nsteps - done, kTabSteps);
        int rc = fill_table(c, c->step + done, chunk, st);
        if (rc != AD_OK) return rc;
        for (int q = 0; q < chunk;) {
            /* steps left before the next record point or the chunk's end */
            long long room = chunk - q;
            if (record_every > 0) room = std::min<long long>(room, record_every - (done + q) % record_every);
            if (resident) {
                /* every step of the run in one launch */
                const long long n0 = c->step + done + q;
                double s0, c0;
                trig_at(c, c->t0 + (double)n0 * c->p.dt, &s0, &c0);
                rc = launch_resident_timed(c, n0, (int)room, s0, c0, st);
                if (rc != AD_OK) return rc;
                q += (int)room;
            } else if (graph) {
                int g = 0;
                while (kGraphSteps[g] > room) ++g; /* the last graph is one step */
                HIPCHECK(c, hipGraphLaunch(c->graph_exec[g], st));
                q += kGraphSteps[g];
            } else {
                rc = launch_step_kernels(c, st);
                if (rc != AD_OK) return rc;
                q += 1;
            }
            const long long n = done + q;
            if (record_every > 0 && n % record_every == 0) {
                double* cp = centres ? centres + rec * 3LL * c->Stot : nullptr;
                double* mp = com ? com + rec * 3LL * c->nsys : nullptr;
                HIPCHECK(c, ad::launch_record(c->dev, cp, mp, st));
                ++rec;
            }
        }
        done += chunk;
    }
    c->step += nsteps;
    /* the resident form keeps its stages in LDS and leaves no pack or step
     * slot behind */
    c->pack_valid = !resident;
    c->slot_valid = !resident;
    return AD_OK;
}

static int read_flag(ad_ctx* c, hipStream_t st) {
    HIPCHECK(c, hipMemcpyAsync(c->h_flag, &c->dev.ctl->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHECK(c, hipStreamSynchronize(st));
    const int f = *c->h_flag;
    if (f & ad::FLAG_NONFINITE) return fail(c, AD_ENONFINITE, "non-finite velocity or coincident spheres met");
    if (f & ad::FLAG_NBR_FULL)
        return fail(c, AD_ERANGE, "more than %d steric candidates for one sphere", ad::NBR_CAP);
    if (f & ad::FLAG_NBR_SKIN) return fail(c, AD_ERANGE, "a sphere moved more than the steric skin allows in one stage");
    return AD_OK;
}

/* ------------------------------------------------------------ ABI */

/* A roctx range over a stepping or mobility call: the host span of the call
 * (its launches and, for ad_run, the flag read) in `rocprofv3 --marker-trace`
 * output, nested under the caller's own ranges. Without a profiler attached
 * a push and a pop cost a few nanoseconds. */
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

extern "C" {

int ad_create(const ad_params* p, int32_t nsys, const int32_t* S_per_sys, ad_ctx** out) {
    g_thread_error[0] = 0;
    if (!p || !S_per_sys || !out) return fail(nullptr, AD_EINVAL, "null argument");
    *out = nullptr;
    if (nsys <= 0) return fail(nullptr, AD_EINVAL, "nsys must be >= 1");
    const double vals[] = {p->a, p->eta, p->k, p->ell, p->lambda, p->T, p->dt, p->steric_k, p->steric_r, p->kT};
    for (double v : vals)
        if (!isfinite(v)) return fail(nullptr, AD_EINVAL, "parameters must be finite");
    if (!(p->a > 0) || !(p->eta > 0) || !(p->T > 0) || !(p->dt > 0))
        return fail(nullptr, AD_EINVAL, "a, eta, T and dt must be > 0");
    if (p->steric_k != 0.0 && !(p->steric_r > 0)) return fail(nullptr, AD_EINVAL, "steric_r must be > 0");
    if (p->precision != AD_FP64 && p->precision != AD_FP64_TILED && p->precision != AD_FP32C &&
        p->precision != AD_FP64_DENSE)
        return fail(nullptr, AD_EINVAL, "unknown precision %d", p->precision);
    if (p->integrator != AD_RK4 && p->integrator != AD_HEUN)
        return fail(nullptr, AD_EINVAL, "unknown integrator %d", p->integrator);
    if (p->tensor != AD_OSEEN && p->tensor != AD_RPY) return fail(nullptr, AD_EINVAL, "unknown tensor %d", p->tensor);
    if (p->reserved != 0) return fail(nullptr, AD_EINVAL, "reserved must be 0");
    if (p->kT < 0.0) return fail(nullptr, AD_EINVAL, "kT must be >= 0");
    if (p->kT > 0.0 && p->integrator != AD_HEUN) return fail(nullptr, AD_EINVAL, "noise (kT > 0) needs AD_HEUN");
    long long Stot = 0;
    for (int b = 0; b < nsys; ++b) {
        if (S_per_sys[b] < 1) return fail(nullptr, AD_EINVAL, "S_per_sys[%d] must be >= 1", b);
        Stot += S_per_sys[b];
    }
    if (2 * Stot > (1LL << 30)) return fail(nullptr, AD_EINVAL, "too many spheres");
    if (p->precision == AD_FP64_DENSE && dense_bytes(nsys, S_per_sys) > kDenseMaxBytes)
        return fail(nullptr, AD_EINVAL, "AD_FP64_DENSE: the pair tensors would take %.3g GB (limit 32 GiB)",
                    dense_bytes(nsys, S_per_sys) / 1e9);
    ad_ctx* c = new (std::nothrow) ad_ctx();
    if (!c) return fail(nullptr, AD_ENOMEM, "out of host memory");
    c->p = *p;
    c->nsys = nsys;
    c->S.assign(S_per_sys, S_per_sys + nsys);
    c->off.assign(nsys + 1, 0);
    for (int b = 0; b < nsys; ++b) c->off[b + 1] = c->off[b] + 2 * c->S[b];
    c->Ntot = c->off[nsys];
    c->Stot = (int)Stot;
    c->dsys.resize(c->Stot);
    for (int b = 0, s = 0; b < nsys; ++b)
        for (int q = 0; q < c->S[b]; ++q) c->dsys[s++] = b;
    c->coef = ad::make_coef(p);
    c->omega = 2.0 * kPi / p->T;
    for (int b = 0; b < nsys; ++b) c->maxNb = std::max(c->maxNb, 2 * c->S[b]);
    c->launch = default_launch(c);
    build_items(c);
    *out = c;
    return AD_OK;
}

int ad_destroy(ad_ctx* c) {
    if (!c) return AD_OK;
    drop_graph(c);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->tab_event) (void)hipEventDestroy(c->tab_event);
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    if (c->h_tab) (void)hipHostFree(c->h_tab);
    if (c->h_phi) (void)hipHostFree(c->h_phi);
    if (c->h_phi_in) (void)hipHostFree(c->h_phi_in);
    if (c->h_flag) (void)hipHostFree(c->h_flag);
    delete c;
    return AD_OK;
}

int ad_workspace_size(const ad_ctx* c, uint64_t* bytes) {
    if (!c || !bytes) return AD_EINVAL;
    *bytes = layout(c).total;
    return AD_OK;
}

int ad_bind_workspace(ad_ctx* c, void* ptr, uint64_t bytes) {
    if (!c) return AD_EINVAL;
    if (!ptr) return fail(c, AD_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(ptr) % 256) return fail(c, AD_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < layout(c).total)
        return fail(c, AD_ENOMEM, "workspace of %llu bytes, need %llu", (unsigned long long)bytes,
                    (unsigned long long)layout(c).total);
    if (!c->h_tab) {
        HIPCHECK(c, hipHostMalloc((void**)&c->h_tab, (size_t)kRing * 8 * sizeof(double), hipHostMallocDefault));
        HIPCHECK(c, hipHostMalloc((void**)&c->h_phi, (size_t)c->Stot * sizeof(double2), hipHostMallocDefault));
        HIPCHECK(c, hipHostMalloc((void**)&c->h_phi_in, (size_t)c->Stot * sizeof(double), hipHostMallocDefault));
        HIPCHECK(c, hipHostMalloc((void**)&c->h_flag, sizeof(int), hipHostMallocDefault));
        HIPCHECK(c, hipEventCreateWithFlags(&c->tab_event, hipEventDisableTiming));
    }
    drop_graph(c);
    c->ws = ptr;
    c->ws_bytes = bytes;
    c->state = false;
    c->pack_valid = false;
    make_dev(c);
    return upload_tables(c);
}

int ad_set_launch(ad_ctx* c, const ad_launch* L) {
    if (!c || !L) return AD_EINVAL;
    ad_launch want = *L;
    ad_launch def = default_launch(c);
    if (want.ipl == 0) want.ipl = def.ipl;
    if (want.wg == 0) want.wg = def.wg;
    if (want.jchunk == 0) want.jchunk = def.jchunk;
    if (want.wj == 0) want.wj = (want.wg == def.wg) ? def.wj : 1;
    if (want.posmode == 0) want.posmode = def.posmode;
    int rc = validate_launch(c, want);
    if (rc != AD_OK) return rc;
    ad_launch old = c->launch;
    c->launch = want;
    build_items(c);
    if (c->ws) {
        if (layout(c).total > c->ws_bytes) {
            c->launch = old;
            build_items(c);
            return fail(c, AD_ENOMEM, "workspace too small for this launch shape");
        }
        /* regions ahead of the work list (state, phases, tables) keep their
         * offsets; the packs, partials and step table move */
        drop_graph(c);
        c->pack_valid = false;
        make_dev(c);
        return upload_tables(c);
    }
    return AD_OK;
}

int ad_get_launch(const ad_ctx* c, ad_launch* L) {
    if (!c || !L) return AD_EINVAL;
    *L = c->launch;
    return AD_OK;
}

int ad_set_state(ad_ctx* c, const double* X, const double* phi, double t0, int64_t step0, void* stream) {
    if (!c) return AD_EINVAL;
    if (!c->ws) return fail(c, AD_ESTATE, "no workspace bound");
    if (!X || !phi) return fail(c, AD_EINVAL, "null X or phi");
    if (!isfinite(t0) || step0 < 0) return fail(c, AD_EINVAL, "t0 must be finite and step0 >= 0");
    hipStream_t st = as_stream(stream);
    /* the phases come to the host once: (sin phi, cos phi) are taken with
     * the host libm, like every sin and cos of the rest length */
    HIPCHECK(c, hipMemcpyAsync(c->h_phi_in, phi, (size_t)c->Stot * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(c, hipStreamSynchronize(st));
    for (int s = 0; s < c->Stot; ++s) {
        const double ph = c->h_phi_in[s];
        if (!isfinite(ph)) return fail(c, AD_EINVAL, "phi[%d] is not finite", s);
        c->h_phi[s] = make_double2(sin(ph), cos(ph));
    }
    HIPCHECK(c, hipMemcpyAsync(const_cast<double2*>(c->dev.phitrig), c->h_phi, (size_t)c->Stot * sizeof(double2),
                               hipMemcpyHostToDevice, st));
    HIPCHECK(c, ad::launch_state_in(c->dev, X, st));
    HIPCHECK(c, ad::launch_clear_flag(c->dev, st));
    HIPCHECK(c, ad::launch_clear_counts(c->dev, st));
    HIPCHECK(c, hipStreamSynchronize(st));
    c->t0 = t0;
    c->step = step0;
    c->state = true;
    c->slot_valid = false;
    c->tab_lo = c->tab_hi = 0; /* the rows depend on t0 */
    c->pack_valid = false;
    return AD_OK;
}

int ad_get_state(ad_ctx* c, double* X, double* t0, int64_t* step, void* stream) {
    if (!c) return AD_EINVAL;
    if (!c->ws || !c->state) return fail(c, AD_ESTATE, "no state loaded");
    hipStream_t st = as_stream(stream);
    if (X) HIPCHECK(c, ad::launch_state_out(c->dev, X, st));
    HIPCHECK(c, hipStreamSynchronize(st));
    if (t0) *t0 = c->t0;
    if (step) *step = c->step;
    return AD_OK;
}

int ad_forces(ad_ctx* c, const double* X, double t, double* F, void* stream) {
    if (!c) return AD_EINVAL;
    const Range range("ad_forces");
    if (!c->ws || !c->state) return fail(c, AD_ESTATE, "no state loaded (phases needed)");
    if (!X || !F) return fail(c, AD_EINVAL, "null X or F");
    if (!isfinite(t)) return fail(c, AD_EINVAL, "t must be finite");
    double s0, c0;
    trig_at(c, t, &s0, &c0);
    HIPCHECK(c, ad::launch_forces(c->dev, c->coef, X, s0, c0, F, as_stream(stream)));
    return AD_OK;
}

int ad_mobility_apply(ad_ctx* c, const double* X, const double* F, double* u, void* stream) {
    if (!c) return AD_EINVAL;
    const Range range("ad_mobility_apply");
    if (!c->ws) return fail(c, AD_ESTATE, "no workspace bound");
    if (!X || !F || !u) return fail(c, AD_EINVAL, "null X, F or u");
    hipStream_t st = as_stream(stream);
    const int prec = prec_of(c);
    c->pack_valid = false; /* the apply pack overwrites the state's */
    HIPCHECK(c, ad::launch_pack_apply(c->dev, c->coef, prec, X, F, st));
    ad::Shape sh = shape_of(c);
    sh.steric = 0; /* candidate lists belong to the step loop */
    const ad::Epi e = epi_of(c, 0, u);
    if (is_dense(c))
        HIPCHECK(c, ad::launch_dense(c->dev, e, 0, c->maxNb, st));
    else
        HIPCHECK(c, ad::launch_pairs(c->dev, e, sh, 0, st));
    HIPCHECK(c, ad::launch_epilogue(c->dev, e, st));
    return AD_OK;
}

int ad_step(ad_ctx* c, int64_t nsteps, void* stream) {
    if (!c) return AD_EINVAL;
    const Range range("ad_step");
    return advance(c, nsteps, 0, nullptr, nullptr, as_stream(stream));
}

int ad_run(ad_ctx* c, int64_t nsteps, int32_t record_every, double* centres, double* com, void* stream) {
    if (!c) return AD_EINVAL;
    if (record_every < 0) return fail(c, AD_EINVAL, "record_every must be >= 0");
    const Range range("ad_run");
    hipStream_t st = as_stream(stream);
    int rc = advance(c, nsteps, record_every, centres, com, st);
    if (rc != AD_OK) return rc;
    return read_flag(c, st);
}

int ad_check(ad_ctx* c, void* stream) {
    if (!c) return AD_EINVAL;
    if (!c->ws) return fail(c, AD_ESTATE, "no workspace bound");
    return read_flag(c, as_stream(stream));
}

int ad_use_graph(ad_ctx* c, int32_t enable) {
    if (!c) return AD_EINVAL;
    c->use_graph = enable != 0;
    return AD_OK;
}

int ad_profile_pairs(ad_ctx* c, int32_t enable) {
    if (!c) return AD_EINVAL;
    if (c->profile && c->ev_used) {
        int rc = profile_flush(c);
        if (rc != AD_OK) return rc;
    }
    c->profile = enable != 0;
    c->prof_ms = 0.0;
    c->prof_launches = 0;
    return AD_OK;
}

int ad_profile_read(ad_ctx* c, double* total_ms, int64_t* launches) {
    if (!c || !total_ms || !launches) return AD_EINVAL;
    int rc = profile_flush(c);
    if (rc != AD_OK) return rc;
    *total_ms = c->prof_ms;
    *launches = c->prof_launches;
    return AD_OK;
}

const char* ad_last_error(const ad_ctx* c) {
    if (!c) return g_thread_error;
    return c->err.c_str();
}

}  // extern "C"
