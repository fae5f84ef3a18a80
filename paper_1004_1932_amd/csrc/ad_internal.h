/*
 * Internal types shared by the kernels (ad_kernels.hip) and the host runtime
 * (ad_runtime.hip). Not part of the ABI.
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ad.h"

namespace ad {

/* One work-group's share of a pair sum: target spheres [i0, i0+ni) against
 * source spheres [j0, j0+nj), both inside system `sys` whose spheres are
 * [ioff, ioff+Nb). `c` numbers the j-chunk inside the system; the partial
 * sum lands in partial slot c of the system. */
struct Item {
    int32_t sys, i0, ni, j0, nj, c, Nb, ioff;
};

/* Device control block at the start of the workspace. */
struct Ctl {
    /* step index as seen by even (slot 0) and odd (slot 1) stages: stage 0
     * copies slot 0 into slot 1, the last stage stores slot 1 + 1 into slot
     * 0, so no kernel reads a slot that it writes */
    long long slot[2];
    int flag; /* FLAG_* bits, sticky until cleared */
    int pad[11];
    /* (sin, cos) of omega t at which stage s's epilogue forms the next
     * forces, copied from the step table by stage s's first kernel, so the
     * epilogue reads it without first reading the step index */
    double trig[4][2];
};

enum {
    FLAG_NONFINITE = 1, /* non-finite velocity or coincident spheres */
    FLAG_NBR_FULL = 2,  /* steric candidate list of a sphere overflowed */
    FLAG_NBR_SKIN = 4,  /* a sphere moved more than half the skin in one stage */
};

/* steric candidate lists (FP32C): spheres closer than rc + skin at the
 * previous stage positions, at most NBR_CAP per sphere */
constexpr int NBR_CAP = 16;

/* dense mode: tensor rows per product work item, and the largest j-chunk
 * (its forces are staged in LDS) */
constexpr int DENSE_ROWS = 256;
constexpr int DENSE_JMAX = 1024;

/* Constants of the model, precomputed on the host. */
struct Coef {
    double cs;   /* 1/(6 pi eta a) */
    double co;   /* 1/(8 pi eta) */
    double k;    /* spring constant */
    double ell;  /* mean length */
    double lam;  /* stroke amplitude */
    double dt;   /* step */
    double h2;   /* 0.5*dt */
    double dt6;  /* dt/6.0 */
    double ks;   /* steric strength (0: off) */
    double rc;   /* steric contact distance */
    double cr;   /* 2 a^2/(24 pi eta): Rotne-Prager-Yamakawa-Mazur coefficient */
    float crr;   /* cr / co = 2 a^2 / 3, for the FP32 pair sum */
    double crr64; /* the same in FP64, for the FP64 streamed stage */
    int rpy;     /* 1: Oseen plus the RPY-Mazur correction; 0: Oseen */
    int noise;   /* 1: Heun with additive noise */
    double g;    /* noise amplitude sqrt(2 kT dt/(6 pi eta a)) */
    unsigned long long seed; /* noise key */
};

/* Device views into the workspace. */
struct Dev {
    Ctl* ctl;
    double* X;          /* [3][Ntot] state, SoA */
    double* R;          /* [3][Ntot] RK accumulator */
    double* U0;         /* [3][Ntot] self (+partner) velocity of the stage */
    double* Y;          /* [3][Ntot] stage positions (steric path only) */
    double* Fs;         /* [3][Ntot] stage forces (steric path only) */
    int* nbr_cnt;       /* [Ntot] candidate count (FP32C steric path) */
    int* nbr_idx;       /* [Ntot][NBR_CAP] candidate source spheres */
    float list_r2;      /* (rc + skin)^2: pairs closer than this are listed */
    double move2;       /* (skin/2)^2: largest allowed stage displacement squared */
    const double2* phitrig; /* [Stot] (sin phi, cos phi) */
    const int* dsys;    /* [Stot] system of each dumbbell */
    const int* sys_off; /* [nsys+1] sphere offsets */
    const int* sys_P;   /* [nsys] number of j-chunks (partial slots) */
    const long long* sys_pbase; /* [nsys] first partial of the system */
    const Item* items;  /* [nitems] */
    float4* pA;         /* FP32C pack read by this stage: (hi.x, hi.y, hi.z, F.x) */
    float4* pB;         /* FP32C pack: (lo.x, lo.y, lo.z, F.y) */
    float2* pC;         /* FP32C pack: (F.y, F.z) */
    double2* pD;        /* FP64 pack: 3 double2 per sphere (x,y)(z,Fx)(Fy,Fz) */
    float4* pA2;        /* the packs the epilogue writes for the next stage */
    float4* pB2;
    float2* pC2;
    double2* pD2;
    double* part;       /* partial sums */
    double* H;          /* dense mode: per system the 3Nb x 3Nb pair tensor, column-major */
    const Item* fitems; /* fused stages of an ensemble: (system, target block) items; the
                           resident form: one per system; AD_FP64 pair sum: target blocks */
    int nfitems;        /* 0: one system, blocks in order */
    const long long* sys_hbase; /* [nsys] dense mode: first element of the system's tensor */
    const double* tab;  /* [ring][8] (sin, cos) of omega*t per epilogue stage */
    int ring;           /* entries in tab, a power of two (rows are step & (ring - 1)) */
    int Ntot, Stot, nsys, nitems;
    int ncomp; /* partial-sum components per sphere: 3, or 6 for FP64 with RPY
                  (Oseen and correction summed apart, as the plain sum does) */
};

enum { PREC_FP64 = 0, PREC_FP64_TILED = 1, PREC_FP32C = 2 };

/* What the epilogue of a stage does. */
struct Epi {
    Coef c;
    int prec;       /* PREC_* */
    int integ;      /* 0 = RK4, 1 = Heun */
    int stage;      /* stage index inside the step */
    int nst;        /* stages per step */
    int pack_next;  /* 1: write the next pack; 0: stage positions and spring forces for the steric kernel */
    double* u_aos;  /* mobility apply: velocities out, row-major [N][3]; else nullptr */
};

/* Step bookkeeping, done by the first kernel of every stage (block 0,
 * thread 0): stage 0 copies slot 0 into slot 1, the last stage advances slot
 * 0; readers in the same stage read the other slot. It also copies the
 * stage's (sin, cos)(omega t) row of the step table into ctl->trig. */
__device__ __forceinline__ void advance_slots(const Dev& d, const Epi& e) {
    if (blockIdx.x != 0 || blockIdx.y != 0 || threadIdx.x != 0) return;
    long long step;
    if (e.stage == 0) {
        step = d.ctl->slot[0];
        d.ctl->slot[1] = step;
    } else {
        step = d.ctl->slot[1];
    }
    if (e.stage == e.nst - 1) d.ctl->slot[0] = step + 1;
    const long long row = step & (d.ring - 1);
    d.ctl->trig[e.stage][0] = d.tab[row * 8 + 2 * e.stage];
    d.ctl->trig[e.stage][1] = d.tab[row * 8 + 2 * e.stage + 1];
}

/* Launch shape of the pair kernel: WG threads = (WG/64/wj) waves on distinct
 * targets x wj waves splitting each j-tile; ipl targets per lane; split = 1
 * for hi/lo positions (FP32C only). One work item covers 64*ipl*WG/64/wj
 * target spheres. */
struct Shape {
    int wg, wj, ipl, split;
    int fused;  /* 0: pair kernel + epilogue; 1: stage kernel, 16 targets per
                   work-group; 2: stage kernel, 64 targets per work-group; 3:
                   stage kernel, 16 targets, sources streamed per wave; 4:
                   resident, one work-group per system for a run of steps */
    int rpy;    /* pair tensor with the RPY-Mazur correction */
    int steric; /* FP32C: record steric candidates while summing */
};

/* Default launch shape of the pair kernel (not the dense mode) for nsys
 * systems of at most maxN spheres: FP64 one system-long j-chunk per target
 * block of 64; small or many systems 64-thread groups over 256-source
 * chunks; large single systems 256-thread groups (4 waves splitting every
 * tile in FP32C) and j-chunks that make about 1024 work-groups. */
struct PairShape {
    int ipl, wg, wj, jchunk;
};
__host__ __device__ inline PairShape default_pair_shape(int prec, int nsys, int maxN) {
    PairShape L{1, 64, 1, 256};
    if (prec == PREC_FP64) {
        L.jchunk = maxN;
        return L;
    }
    if (nsys > 1 || maxN < 1024) return L;
    L.wg = 256;
    if (prec == PREC_FP32C) L.wj = 4;
    const int IB = L.ipl * L.wg / L.wj;
    const int blocks = (maxN + IB - 1) / IB;
    const int P = blocks >= 1024 ? 1 : 1024 / blocks;
    int jc = (maxN + P - 1) / P;
    jc = (jc + L.wg - 1) / L.wg * L.wg;
    L.jchunk = jc > L.wg ? jc : L.wg;
    return L;
}

/* host helpers (ad_runtime.hip): the model constants of a parameter set,
 * and the thread's error message of the context-free calls (a fixed
 * buffer; printf-style, returns code) */
Coef make_coef(const ad_params* p);
int thread_fail(int code, const char* fmt, ...);
void thread_clear_error();

/* kernel launchers (ad_kernels.hip) */
hipError_t launch_set_step(const Dev& d, long long step, hipStream_t s);
hipError_t launch_clear_flag(const Dev& d, hipStream_t s);
hipError_t launch_clear_counts(const Dev& d, hipStream_t s);
hipError_t launch_state_in(const Dev& d, const double* Xaos, hipStream_t s);
hipError_t launch_state_out(const Dev& d, double* Xaos, hipStream_t s);
/* pack from the state X at forces time (st, ct), into the first pack */
hipError_t launch_pack_state(const Dev& d, const Coef& c, int prec, double st, double ct, hipStream_t s);
/* pack from caller positions and forces (row-major), into the first pack */
hipError_t launch_pack_apply(const Dev& d, const Coef& c, int prec, const double* Xaos,
                             const double* Faos, hipStream_t s);
/* forces at caller positions (row-major) and time (st, ct), spring + steric */
hipError_t launch_forces(const Dev& d, const Coef& c, const double* Xaos, double st, double ct,
                         double* Faos, hipStream_t s);
/* pair sum; mode 0 = mobility apply, 1 = step stage. With events, they time
 * the dispatch itself. */
hipError_t launch_pairs(const Dev& d, const Epi& e, const Shape& sh, int mode, hipStream_t s,
                        hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
/* dense mode (ad_dense.hip): assemble every system's pair tensor from the
 * FP64 pack, then multiply it by the packed forces into the partial sums;
 * the events, if given, bracket both launches */
hipError_t launch_dense(const Dev& d, const Epi& e, int mode, int maxNb, hipStream_t s,
                        hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
/* FP32C without steric forces: pair sum and epilogue of a stage in one
 * kernel, every source of a work-group's system in LDS (at most
 * FUSED_LDS_MAX bytes: 6784 spheres per system with single-float, 4544 with
 * hi/lo positions); 16 waves per work-group for one system, 4 waves and the
 * work list fitems for an ensemble */
constexpr int FUSED_LDS_MAX = 160 * 1024; /* the kernel has no static LDS */
/* LDS bytes of a fused work-group for a system of n spheres: the sources,
 * padded to the 4 nw source splits (36 B each with hi/lo positions, 24 B
 * with single-float), or the combination area it reuses (nw waves x 16
 * targets x 6 floats, 16 x 3 stage positions) if larger */
__host__ __device__ inline int fused_lds_bytes(int n, int split, int nw) {
    const int js = 4 * nw;
    const int np = (n + js - 1) / js * js;
    const int b = np * (split ? 36 : 24);
    const int red = nw * 16 * 6 * 4 + 16 * 3 * 8;
    return b > red ? b : red;
}
/* LDS bytes of a wide fused work-group (64 targets, 4 waves): the sources
 * padded to 4, or the combination area (4 waves x 64 targets x 6 floats,
 * 64 x 3 stage positions, a flag) if larger */
constexpr int FW_I = 64;
__host__ __device__ inline int fused_wide_lds_bytes(int n, int split) {
    const int np = (n + 3) / 4 * 4;
    const int b = np * (split ? 36 : 24);
    const int red = 4 * FW_I * 6 * 4 + FW_I * 3 * 8 + 16;
    return b > red ? b : red;
}
/* AD_FP64 pair sum with producer and consumer waves (k_pairs_f64w):
 * producer waves per work-group (one, two and three measured at N = 512 to
 * 8192: one was fastest everywhere, by 4 to 12 %); targets per work-group,
 * about Ntot / 1024 from 1 to 4, so that the launch holds about two waves per
 * SIMD; sources per chunk: 128 where a launch of 4-target work-groups holds
 * at most one producer wave per SIMD (Ntot below 8192: 7 % faster at 4096,
 * more independent terms per lane), else 64 (at 8192 the larger chunk's
 * registers cost a wave per SIMD, 48 % slower) */
constexpr int F64W_NP = 1;
__host__ __device__ inline int f64w_targets(int Ntot) { return Ntot >= 4096 ? 4 : Ntot >= 2048 ? 2 : 1; }
__host__ __device__ inline int f64w_chunk(int Ntot) { return f64w_targets(Ntot) == 4 && Ntot < 8192 ? 128 : 64; }
/* LDS of a work-group: two sets of F64W_NP chunk buffers of rows x (cw + 1) */
__host__ __device__ inline int f64w_lds_bytes(int tw, int rpy, int cw) {
    return 2 * F64W_NP * (rpy ? 6 : 3) * tw * (cw + 1) * 8;
}
/* the most target spheres per work-group of the streamed fused stage */
constexpr int FT_I = 16;
/* target spheres per work-group of the streamed fused stage for Ntot
 * spheres in all: 4, 8 or 16, about Ntot / 256, so that the launch holds
 * about one work-group per compute unit (every work-group reads every source
 * of its system: two on a compute unit double that traffic; fewer than 256
 * leave compute units idle) */
__host__ __device__ inline int stream_targets(int Ntot) {
    int ti = 4;
    while (ti < FT_I && 2 * 256 * ti <= Ntot) ti *= 2;
    return ti;
}
/* waves per work-group of the streamed fused stage with ti targets: 16 with
 * 16 targets, else 8. With 4 targets (the small systems) the few sources per
 * lane make the combination of 16 waves' sums a large share; with 8 targets
 * (2048 to 4095 spheres) an 8-wave work-group lets two share a compute unit
 * when the launch has more than 256 (N = 3072: 42.1 against 49.0 us per
 * step; N = 2048 equal) */
__host__ __device__ inline int stream_waves(int ti) { return ti == 16 ? 16 : 8; }
/* LDS bytes of a streamed fused work-group: nw waves x 2 slots x 64 source
 * entries, followed by the combination area (nw waves x ti targets x 6
 * floats, ti x 3 stage positions); at most 16 waves and 16 targets */
__host__ __device__ inline int fused_stream_lds_bytes(int split, int nw = 16, int ti = FT_I) {
    const int b = nw * 2 * 64 * (split ? 36 : 24);
    const int red = nw * ti * 6 * 4 + ti * 3 * 8;
    return b + red;
}
/* LDS bytes of an FP64 streamed work-group: 16 waves x 2 slots x 64 source
 * entries of 48 B, then the combination area (16 waves x at most 16 targets x
 * 3 doubles, 16 x 3 stage positions) */
__host__ __device__ inline int fused_stream64_lds_bytes() { return 16 * 2 * 64 * 48 + 16 * 16 * 3 * 8 + 16 * 3 * 8; }
/* Resident form (launch.fused = 4): one work-group of RES_T threads per
 * system holds the whole system in LDS and runs every stage of a run of
 * steps in one launch. Systems of at most RES_MAX64 spheres with FP64 pair
 * sums, RES_MAX32 with FP32C. */
constexpr int RES_T = 256;
constexpr int RES_MAX64 = 128;
constexpr int RES_MAX32 = 256;
/* FP64 term-matrix budget per column chunk */
constexpr int RES_TERM_BYTES = 64 * 1024;
/* dynamic LDS a resident work-group may use (the largest need is 84 KiB:
 * 128 FP64 spheres with RPY); the kernels also hold a little static LDS */
constexpr int RES_LDS_MAX = 96 * 1024;
/* source columns of one FP64 term-matrix chunk for a system of n spheres */
__host__ __device__ inline int resident_cols(int n, int rpy) {
    const int per = n * 24 * (rpy ? 2 : 1);
    int cc = RES_TERM_BYTES / (per > 0 ? per : 1);
    if (cc < 1) cc = 1;
    return cc < n ? cc : n;
}
/* LDS row stride (doubles) of an FP64 term chunk of cc columns: odd */
__host__ __device__ inline int resident_col_stride(int cc) { return cc | 1; }
/* float4 entries of one FP32C resident pack buffer: A = (hi.xyz, Fx) and
 * B = (lo.xyz, Fy) per sphere, then Fz per sphere */
__host__ __device__ inline int resident_pack_f4(int n) { return 2 * n + (n + 3) / 4; }
/* LDS bytes of a resident work-group for a system of n spheres: FP64 holds
 * X, R, Y and F (3n doubles each) and the pair sums (3n, twice with RPY),
 * then the term-matrix chunk; FP32C keeps its state in registers and holds
 * two pack buffers */
__host__ __device__ inline int resident_lds_bytes(int n, int p64, int rpy) {
    if (!p64) return 2 * resident_pack_f4(n) * 16;
    const int b = (3 * n * (5 + (rpy ? 1 : 0)) * 8 + 15) / 16 * 16;
    return b + resident_col_stride(resident_cols(n, rpy)) * n * 24 * (rpy ? 2 : 1);
}
/* threads of a resident work-group: FP64 RES_T (its term evaluations are
 * long dependent chains, best spread over the four SIMDs); FP32C one wave up
 * to 16 spheres (its barriers cost next to nothing), above that the smallest
 * power of two up to 512 with 8 lanes per sphere of the largest system (4
 * lanes measured slower from 32 to 64 spheres, 8 lanes over two waves
 * slower at 16) */
__host__ __device__ inline int resident_threads(int maxn, int p64) {
    if (p64) return RES_T;
    if (maxn <= 16) return 64;
    int t = 128;
    while (t < 512 && t < 8 * maxn) t *= 2;
    return t;
}
/* lanes per target sphere in the FP32C resident pair sum: the largest power
 * of two s <= 32 with s n <= t (t threads); at most 32, so the lanes of both
 * spheres of a dumbbell lie in one wave */
__host__ __device__ inline int resident_split(int n, int t) {
    int s = 1;
    while (s < 32 && 2 * s * n <= t) s *= 2;
    return s;
}
hipError_t launch_resident(const Dev& d, const Epi& e, int hilo, int maxNb, long long step0, int nsteps,
                           double st0, double ct0, hipStream_t s, hipEvent_t ev_start = nullptr,
                           hipEvent_t ev_stop = nullptr);

/* allow the fused kernels FUSED_LDS_MAX bytes of dynamic LDS (host call,
 * outside any stream capture) */
hipError_t prepare_fused();
hipError_t launch_fused(const Dev& d, const Epi& e, const Shape& sh, int maxNb, hipStream_t s,
                        hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
hipError_t launch_epilogue(const Dev& d, const Epi& e, hipStream_t s);
/* steric forces at stage positions Y, then the next pack (steric path) */
hipError_t launch_steric_pack(const Dev& d, const Coef& c, int prec, hipStream_t s);
hipError_t launch_record(const Dev& d, double* centres, double* com, hipStream_t s);

}  // namespace ad
