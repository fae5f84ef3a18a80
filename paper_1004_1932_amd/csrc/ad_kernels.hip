/*
 * HIP kernels for gfx950 (CDNA4): the all-pairs Oseen mobility step of
 * active spring dumbbell suspensions (Putz, Dunkel, Yeomans, Sec. II and
 * Sec. V).
 *
 * One RK4 stage is two launches:
 *   k_pairs_*   the O(N^2) pair sum over a work list of (i-block, j-chunk)
 *               items; each item stages its j-tiles through LDS and every
 *               lane holds IPL consecutive target spheres in registers.
 *   k_epilogue  sums the j-chunk partials in chunk order, forms the stage
 *               velocity k = u0 + kappa*acc, updates the RK accumulator and
 *               the state, and evaluates the spring forces of the next stage
 *               (Eq. e:swimmer_potential) into the pack the next pair sum
 *               reads.
 * Packs are double-buffered: stage s reads one and writes the other.
 *
 * All FP64 arithmetic is written in a fixed order and built without FMA
 * contraction; FP32 FMAs are spelled out with __builtin_fmaf.
 */
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "ad_internal.h"

namespace ad {

/* ------------------------------------------------------------ helpers */

__device__ __forceinline__ void spring_forces(const Coef& c, const double y0[3], const double y1[3],
                                              double sphi, double cphi, double st, double ct,
                                              double f0[3], double f1[3]) {
    /* F_{2s+1} = -k (d - L) n/d, F_{2s} = -F_{2s+1}, n = y1 - y0,
     * L = ell + lam sin(omega t + phi) by the addition theorem. */
    double nx = y1[0] - y0[0], ny = y1[1] - y0[1], nz = y1[2] - y0[2];
    double d = sqrt((nx * nx + ny * ny) + nz * nz);
    double L = c.ell + c.lam * (st * cphi + ct * sphi);
    double cc = (-c.k * (d - L)) / d;
    f1[0] = cc * nx;
    f1[1] = cc * ny;
    f1[2] = cc * nz;
    f0[0] = -f1[0];
    f0[1] = -f1[1];
    f0[2] = -f1[2];
}

/* Oseen term of one source sphere in FP64, without the 1/(8 pi eta) factor:
 * [F/r + r (r.F)/r^3]. */
__device__ __forceinline__ void oseen_term64(const double r[3], const double F[3], double out[3]) {
    double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    double ir = 1.0 / sqrt(r2);
    double fr = (r[0] * F[0] + r[1] * F[1]) + r[2] * F[2];
    double t = fr / r2;
    out[0] = ir * (F[0] + t * r[0]);
    out[1] = ir * (F[1] + t * r[1]);
    out[2] = ir * (F[2] + t * r[2]);
}

/* Rotne-Prager-Yamakawa-Mazur correction of one source sphere in FP64,
 * without its 2a^2/(24 pi eta) factor: (F - 3 r (r.F)/r^2)/r^3, in the
 * operation order of the plain sum. */
__device__ __forceinline__ void rpy_term64(const double r[3], const double F[3], double out[3]) {
    double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    double ir = 1.0 / sqrt(r2);
    double fr = (r[0] * F[0] + r[1] * F[1]) + r[2] * F[2];
    double t = fr / r2;
    double ir3 = ir / r2;
    double t3 = 3.0 * t;
    out[0] = ir3 * (F[0] - t3 * r[0]);
    out[1] = ir3 * (F[1] - t3 * r[1]);
    out[2] = ir3 * (F[2] - t3 * r[2]);
}

/* Steric sum for sphere i over the spheres [j0, j1) of its system: for
 * 0 < r < rc, ks (rc - r) (X_i - X_j)/r, ascending j. Positions are read
 * through `get`. Returns non-zero if a coincident sphere was met. */
template <class Get>
__device__ int steric_sum(const Coef& c, int i, int j0, int j1, Get get, double acc[3], int* any) {
    double xi[3];
    get(i, xi);
    double rc2 = c.rc * c.rc;
    int bad = 0;
    acc[0] = acc[1] = acc[2] = 0.0;
    *any = 0;
    for (int j = j0; j < j1; ++j) {
        if (j == i) continue;
        double xj[3];
        get(j, xj);
        double rx = xi[0] - xj[0], ry = xi[1] - xj[1], rz = xi[2] - xj[2];
        double r2 = (rx * rx + ry * ry) + rz * rz;
        if (r2 >= rc2) continue;
        if (r2 == 0.0) {
            bad = 1;
            continue;
        }
        double r = sqrt(r2);
        double cc = c.ks * (c.rc - r) / r;
        acc[0] = acc[0] + cc * rx;
        acc[1] = acc[1] + cc * ry;
        acc[2] = acc[2] + cc * rz;
        *any = 1;
    }
    return bad;
}

__device__ __forceinline__ void split_f32(double v, float& hi, float& lo) {
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

/* (hi, lo) += v with TwoSum: hi + lo keeps the exact sum up to the rounding
 * of lo. */
__device__ __forceinline__ void two_sum_acc(float& hi, float& lo, float v) {
    const float s = hi + v;
    const float bb = s - hi;
    const float e = (hi - (s - bb)) + (v - bb);
    hi = s;
    lo = lo + e;
}


/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 32x32->64 multiplications by the published multipliers, the key bumped by
 * the Weyl constants between rounds. */
__device__ __forceinline__ void philox4x32_10(unsigned c[4], unsigned k0, unsigned k1) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const unsigned hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const unsigned hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const unsigned n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

/* Standard normal component a (0..2) of sphere i at step n: Box-Muller on
 * the four uniforms (x + 1/2) 2^-32 of one Philox block with counter
 * (i, n) and key seed. */
__device__ double gauss_component(unsigned long long seed, int i, long long n, int a) {
    unsigned c[4] = {(unsigned)i, (unsigned)n, (unsigned)((unsigned long long)n >> 32), 0u};
    philox4x32_10(c, (unsigned)seed, (unsigned)(seed >> 32));
    const double two_pi = 2.0 * 3.14159265358979323846;
    const int pr = (a == 2) ? 2 : 0;
    const double u0 = ((double)c[pr] + 0.5) / 4294967296.0;
    const double u1 = ((double)c[pr + 1] + 0.5) / 4294967296.0;
    const double rr = sqrt(-2.0 * log(u0));
    return (a == 1) ? rr * sin(two_pi * u1) : rr * cos(two_pi * u1);
}

/* Write the pair-kernel pack and the self (+partner) velocity u0 of the two
 * spheres of one dumbbell at positions y0, y1 with forces f0, f1; into the
 * next-stage pack buffers when nxt != 0. */
/* FP32C pack of sphere i at stage position y with spring force f, its
 * dumbbell partner at yp with force fp: u0 = self term plus the partner's
 * term in FP64 (the pair kernels skip the partner), then the FP32 hi/lo
 * position and force: A = (hi.xyz, Fx), B = (lo.xyz, Fy), C = (Fy, Fz), so
 * that a reader of single-float positions needs A and C only. */
__device__ __forceinline__ void store_pack_sphere(const Dev& d, const Coef& c, int i, const double y[3],
                                                  const double yp[3], const double f[3], const double fp[3],
                                                  int nxt) {
    const int N = d.Ntot;
    const double r[3] = {y[0] - yp[0], y[1] - yp[1], y[2] - yp[2]};
    double t[3], q[3];
    oseen_term64(r, fp, t);
    if (c.rpy) rpy_term64(r, fp, q);
    for (int a = 0; a < 3; ++a) {
        double u = c.cs * f[a] + c.co * t[a];
        if (c.rpy) u = u + c.cr * q[a];
        d.U0[a * N + i] = u;
    }
    float h[3], l[3];
    for (int a = 0; a < 3; ++a) split_f32(y[a], h[a], l[a]);
    (nxt ? d.pA2 : d.pA)[i] = make_float4(h[0], h[1], h[2], (float)f[0]);
    (nxt ? d.pB2 : d.pB)[i] = make_float4(l[0], l[1], l[2], (float)f[1]);
    (nxt ? d.pC2 : d.pC)[i] = make_float2((float)f[1], (float)f[2]);
}

/* The closing update of the FP32C stage kernels uses these two forms of
 * spring_forces and store_pack_sphere: one rsqrt (a few ulp) in place of
 * each IEEE sqrt and division. In the FP32C path the state stays FP64 and
 * only the pair sums are FP32, so a relative error near 1e-16 here is far
 * below theirs (about 1e-7); the FP64 paths keep the IEEE forms, whose
 * operation order the bitwise parity with the plain sum depends on. With
 * single-float positions (SPLIT = 0) no stage kernel reads the lo parts, so
 * B is not written. spring_forces_rs returns the 1/d it used. */
__device__ __forceinline__ double spring_forces_rs(const Coef& c, const double y0[3], const double y1[3],
                                                   double sphi, double cphi, double st, double ct,
                                                   double f0[3], double f1[3]) {
    /* -k (d - L) n / d = k (L / d - 1) n */
    const double nx = y1[0] - y0[0], ny = y1[1] - y0[1], nz = y1[2] - y0[2];
    const double id = rsqrt((nx * nx + ny * ny) + nz * nz);
    const double L = c.ell + c.lam * (st * cphi + ct * sphi);
    const double cc = c.k * (L * id - 1.0);
    f1[0] = cc * nx;
    f1[1] = cc * ny;
    f1[2] = cc * nz;
    f0[0] = -f1[0];
    f0[1] = -f1[1];
    f0[2] = -f1[2];
    return id;
}

template <int SPLIT>
__device__ __forceinline__ void store_pack_sphere_rs(const Dev& d, const Coef& c, int i, const double y[3],
                                                     const double yp[3], const double f[3], const double fp[3]) {
    const int N = d.Ntot;
    const double r[3] = {y[0] - yp[0], y[1] - yp[1], y[2] - yp[2]};
    const double ir = rsqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
    const double ir2 = ir * ir;
    const double t = ((r[0] * fp[0] + r[1] * fp[1]) + r[2] * fp[2]) * ir2;
    for (int a = 0; a < 3; ++a) {
        double u = c.cs * f[a] + c.co * (ir * (fp[a] + t * r[a]));
        if (c.rpy) u = u + c.cr * ((ir * ir2) * (fp[a] - (3.0 * t) * r[a]));
        d.U0[a * N + i] = u;
    }
    float h[3], l[3];
    for (int a = 0; a < 3; ++a) split_f32(y[a], h[a], l[a]);
    d.pA2[i] = make_float4(h[0], h[1], h[2], (float)f[0]);
    if (SPLIT) d.pB2[i] = make_float4(l[0], l[1], l[2], (float)f[1]);
    d.pC2[i] = make_float2((float)f[1], (float)f[2]);
}

__device__ void store_pack(const Dev& d, const Coef& c, int prec, int i0, const double y0[3],
                           const double y1[3], const double f0[3], const double f1[3], int nxt) {
    const int N = d.Ntot;
    const int i1 = i0 + 1;
    if (prec == PREC_FP32C) {
        store_pack_sphere(d, c, i0, y0, y1, f0, f1, nxt);
        store_pack_sphere(d, c, i1, y1, y0, f1, f0, nxt);
    } else {
        for (int a = 0; a < 3; ++a) {
            d.U0[a * N + i0] = c.cs * f0[a];
            d.U0[a * N + i1] = c.cs * f1[a];
        }
        double2* pD = nxt ? d.pD2 : d.pD;
        pD[3 * i0 + 0] = make_double2(y0[0], y0[1]);
        pD[3 * i0 + 1] = make_double2(y0[2], f0[0]);
        pD[3 * i0 + 2] = make_double2(f0[1], f0[2]);
        pD[3 * i1 + 0] = make_double2(y1[0], y1[1]);
        pD[3 * i1 + 1] = make_double2(y1[2], f1[0]);
        pD[3 * i1 + 2] = make_double2(f1[1], f1[2]);
    }
}

/* ------------------------------------------------------------ small kernels */

__global__ void k_set_step(Ctl* ctl, long long v) { ctl->slot[0] = v; }
__global__ void k_clear_flag(Ctl* ctl) { ctl->flag = 0; }

__global__ void k_state_in(Dev d, const double* __restrict__ Xa) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.Ntot) return;
    for (int a = 0; a < 3; ++a) d.X[a * d.Ntot + i] = Xa[3 * i + a];
}

__global__ void k_state_out(Dev d, double* __restrict__ Xa) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.Ntot) return;
    for (int a = 0; a < 3; ++a) Xa[3 * i + a] = d.X[a * d.Ntot + i];
}

/* empty every steric candidate list */
__global__ void k_clear_counts(Dev d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.Ntot || !d.nbr_cnt) return;
    d.nbr_cnt[i] = 0;
}

/* pack from the state at time (st, ct); spring (+ steric) forces */
__global__ void k_pack_state(Dev d, Coef c, int prec, double st, double ct) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.Stot) return;
    const int N = d.Ntot;
    const int i0 = 2 * s;
    double y0[3], y1[3], f0[3], f1[3];
    for (int a = 0; a < 3; ++a) {
        y0[a] = d.X[a * N + i0];
        y1[a] = d.X[a * N + i0 + 1];
    }
    double2 tp = d.phitrig[s];
    spring_forces(c, y0, y1, tp.x, tp.y, st, ct, f0, f1);
    if (c.ks != 0.0) {
        int b = d.dsys[s];
        int j0 = d.sys_off[b], j1 = d.sys_off[b + 1];
        auto get = [&](int j, double x[3]) {
            x[0] = d.X[j];
            x[1] = d.X[N + j];
            x[2] = d.X[2 * N + j];
        };
        double acc[3];
        int any, bad = 0;
        bad |= steric_sum(c, i0, j0, j1, get, acc, &any);
        if (any)
            for (int a = 0; a < 3; ++a) f0[a] = f0[a] + acc[a];
        bad |= steric_sum(c, i0 + 1, j0, j1, get, acc, &any);
        if (any)
            for (int a = 0; a < 3; ++a) f1[a] = f1[a] + acc[a];
        if (bad) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
        /* stage positions (for the displacement check) and empty candidate
         * lists for the first pair sum */
        for (int a = 0; a < 3; ++a) {
            d.Y[a * N + i0] = y0[a];
            d.Y[a * N + i0 + 1] = y1[a];
        }
        if (d.nbr_cnt) {
            d.nbr_cnt[i0] = 0;
            d.nbr_cnt[i0 + 1] = 0;
        }
    }
    store_pack(d, c, prec, i0, y0, y1, f0, f1, 0);
}

/* pack from caller positions and forces (row-major [N][3]) */
__global__ void k_pack_apply(Dev d, Coef c, int prec, const double* __restrict__ Xa,
                             const double* __restrict__ Fa) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.Stot) return;
    const int i0 = 2 * s;
    double y0[3], y1[3], f0[3], f1[3];
    for (int a = 0; a < 3; ++a) {
        y0[a] = Xa[3 * i0 + a];
        y1[a] = Xa[3 * i0 + 3 + a];
        f0[a] = Fa[3 * i0 + a];
        f1[a] = Fa[3 * i0 + 3 + a];
    }
    store_pack(d, c, prec, i0, y0, y1, f0, f1, 0);
}

/* spring + steric forces at caller positions, row-major output */
__global__ void k_forces(Dev d, Coef c, const double* __restrict__ Xa, double st, double ct,
                         double* __restrict__ Fa) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.Stot) return;
    const int i0 = 2 * s;
    double y0[3], y1[3], f0[3], f1[3];
    for (int a = 0; a < 3; ++a) {
        y0[a] = Xa[3 * i0 + a];
        y1[a] = Xa[3 * i0 + 3 + a];
    }
    double2 tp = d.phitrig[s];
    spring_forces(c, y0, y1, tp.x, tp.y, st, ct, f0, f1);
    if (c.ks != 0.0) {
        int b = d.dsys[s];
        int j0 = d.sys_off[b], j1 = d.sys_off[b + 1];
        auto get = [&](int j, double x[3]) {
            x[0] = Xa[3 * j];
            x[1] = Xa[3 * j + 1];
            x[2] = Xa[3 * j + 2];
        };
        double acc[3];
        int any, bad = 0;
        bad |= steric_sum(c, i0, j0, j1, get, acc, &any);
        if (any)
            for (int a = 0; a < 3; ++a) f0[a] = f0[a] + acc[a];
        bad |= steric_sum(c, i0 + 1, j0, j1, get, acc, &any);
        if (any)
            for (int a = 0; a < 3; ++a) f1[a] = f1[a] + acc[a];
        if (bad) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
    }
    for (int a = 0; a < 3; ++a) {
        Fa[3 * i0 + a] = f0[a];
        Fa[3 * i0 + 3 + a] = f1[a];
    }
}

/* ------------------------------------------------------------ epilogue */

/* Stage update of one state component o = a N + i from its velocity k:
 * RK4 keeps the weighted sum of the stage velocities in R and writes X at the
 * last stage; Heun adds the same noise in both stages. Returns the position
 * at which the next stage evaluates the velocity. */
__device__ __forceinline__ double stage_update(const Dev& d, const Epi& e, int o, int i, int a, double k,
                                               double x, double r, long long step) {
    const Coef& c = e.c;
    const int stage = e.stage;
    double y;
    if (e.integ == 0) { /* RK4 */
        if (stage == 0) {
            d.R[o] = k;
            y = x + c.h2 * k;
        } else if (stage == 1) {
            d.R[o] = r + 2.0 * k;
            y = x + c.h2 * k;
        } else if (stage == 2) {
            d.R[o] = r + 2.0 * k;
            y = x + c.dt * k;
        } else {
            y = x + c.dt6 * (r + k);
            d.X[o] = y;
        }
    } else { /* Heun, with the same noise in both stages */
        const double nz = c.noise ? c.g * gauss_component(c.seed, i, step, a) : 0.0;
        if (stage == 0) {
            d.R[o] = k;
            y = x + c.dt * k;
        } else {
            y = x + c.h2 * (r + k);
        }
        if (c.noise) y = y + nz;
        if (stage == 1) d.X[o] = y;
    }
    return y;
}

constexpr int EPI_MAXP = 16; /* partials loaded per batch */

/* Epilogue of the spheres [i0, i0 + ni) (ni even), run by all blockDim.x
 * threads of a work-group.
 * Phase 1, one thread per sphere component: issue the loads of that
 * component's j-chunk partials, u0, X and R together, sum the partials in
 * chunk order, form k = u0 + kappa*acc and apply the (componentwise) RK
 * update: R, X to global memory, the next stage position y to LDS.
 * Phase 2, one thread per dumbbell: the next stage's spring forces at y and
 * the next pack (or, with steric forces, y and the spring forces for the
 * steric kernel). `step` numbers the noise of the Heun integrator; ys and
 * mv are LDS scratch of ni x 3 doubles. */
__device__ void epi_block(const Dev& d, const Epi& e, int i0, int ni, long long step, double (*ys)[3],
                          double (*mv)[3], int* badf) {
    const int N = d.Ntot;
    const int t = threadIdx.x;
    const int nt = blockDim.x;
    const Coef& c = e.c;
    const int stage = e.stage;
    const bool apply = (e.u_aos != nullptr);
    /* the second pass's inputs are loaded first, so their latency overlaps
     * the partial-sum loads: (sin, cos) of omega t for the next stage's
     * forces (left by this stage's pair kernel), and the phase of this
     * thread's dumbbell */
    double st = 0.0, ct = 0.0;
    double2 tp = make_double2(0.0, 0.0);
    if (!apply) {
        st = d.ctl->trig[stage][0];
        ct = d.ctl->trig[stage][1];
        if (t < ni / 2) tp = d.phitrig[(i0 >> 1) + t];
    }
    if (t == 0) *badf = 0;
    __syncthreads();
    for (int idx = t; idx < 3 * ni; idx += nt) {
        const int sl = idx / 3, a = idx - 3 * sl;
        const int i = i0 + sl;
        const int b = d.dsys[i >> 1];
        const int off = d.sys_off[b];
        const int Nb = d.sys_off[b + 1] - off;
        const int P = d.sys_P[b];
        const long long stride = (long long)d.ncomp * Nb;
        const double* p = d.part + d.sys_pbase[b] + (long long)a * Nb + (i - off);
        const int o = a * N + i;
        /* independent loads first, so they are in flight together */
        const double u0 = d.U0[o];
        const double x = apply ? 0.0 : d.X[o];
        const double r = (!apply && stage > 0) ? d.R[o] : 0.0;
        const double yold = (!apply && !e.pack_next && d.nbr_cnt) ? d.Y[o] : 0.0;
        double v[EPI_MAXP];
#pragma unroll
        for (int q = 0; q < EPI_MAXP; ++q) v[q] = (q < P) ? p[q * stride] : 0.0;
        double acc = v[0];
#pragma unroll
        for (int q = 1; q < EPI_MAXP; ++q)
            if (q < P) acc = acc + v[q];
        for (int cc = EPI_MAXP; cc < P; cc += EPI_MAXP) {
#pragma unroll
            for (int q = 0; q < EPI_MAXP; ++q) v[q] = (cc + q < P) ? p[(cc + q) * stride] : 0.0;
#pragma unroll
            for (int q = 0; q < EPI_MAXP; ++q)
                if (cc + q < P) acc = acc + v[q];
        }
        double k = u0 + c.co * acc;
        if (d.ncomp == 6) {
            /* FP64 with RPY: the correction's partial sums follow the Oseen
             * ones, added after them as in the plain sum */
            const double* p2 = p + 3LL * Nb;
            double acc2 = p2[0];
            for (int cc = 1; cc < P; ++cc) acc2 = acc2 + p2[cc * stride];
            k = k + c.cr * acc2;
        }
        if (!isfinite(k)) *badf = 1;
        if (apply) {
            e.u_aos[3 * i + a] = k;
            continue;
        }
        const double y = stage_update(d, e, o, i, a, k, x, r, step);
        ys[sl][a] = y;
        const double dd = y - yold;
        mv[sl][a] = dd * dd;
    }
    __syncthreads();
    if (t == 0 && *badf) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
    if (apply) return;
    /* forces of the next stage, one thread per dumbbell (ni/2 <= blockDim) */
    if (t < ni / 2) {
        const int q = t;
        const int ia = i0 + 2 * q;
        double y[2][3];
        for (int h = 0; h < 2; ++h)
            for (int a = 0; a < 3; ++a) y[h][a] = ys[2 * q + h][a];
        double f0[3], f1[3];
        spring_forces(c, y[0], y[1], tp.x, tp.y, st, ct, f0, f1);
        if (e.pack_next) {
            store_pack(d, c, e.prec, ia, y[0], y[1], f0, f1, 1);
        } else {
            if (d.nbr_cnt) {
                /* candidate lists are valid while no sphere moves more than
                 * half the skin between stage positions */
                for (int h = 0; h < 2; ++h) {
                    const double e2 = (mv[2 * q + h][0] + mv[2 * q + h][1]) + mv[2 * q + h][2];
                    if (!(e2 <= d.move2)) atomicOr(&d.ctl->flag, FLAG_NBR_SKIN);
                }
            }
            for (int a = 0; a < 3; ++a) {
                d.Y[a * N + ia] = y[0][a];
                d.Y[a * N + ia + 1] = y[1][a];
                d.Fs[a * N + ia] = f0[a];
                d.Fs[a * N + ia + 1] = f1[a];
            }
        }
    }
}

/* the epilogue as its own kernel: EPI_S spheres per work-group of EPI_T
 * threads; the step index comes from the slot the pair kernel left for this
 * stage */
constexpr int EPI_S = 32;
constexpr int EPI_T = 96;
static_assert(EPI_S / 2 <= EPI_T, "one thread per dumbbell in the second pass");

__global__ __launch_bounds__(EPI_T) void k_epilogue(Dev d, Epi e) {
    __shared__ double ys[EPI_S][3];
    __shared__ double mv[EPI_S][3];
    __shared__ int badf;
    const int i0 = blockIdx.x * EPI_S;
    const int ni = min(EPI_S, d.Ntot - i0);
    /* the step index only numbers the noise of the Heun integrator */
    const long long step = (e.u_aos || !e.c.noise) ? 0 : d.ctl->slot[e.stage & 1];
    epi_block(d, e, i0, ni, step, ys, mv, &badf);
}

/* ------------------------------------------------------------ pair sums */

/* Accumulate one FP32 pair term given ir = 1/r (0 for a skipped pair):
 * Oseen: ir (F + t r), t = (r.F) ir^2; with RPY (c' = 2a^2/3):
 * F (ir + c' ir^3) + r t (ir - 3 c' ir^3). */
template <int RPY>
__device__ __forceinline__ void pair_term(float ir, float rx, float ry, float rz, float Fx, float Fy, float Fz,
                                          float crr, float& px, float& py, float& pz) {
    const float fr = __builtin_fmaf(rz, Fz, __builtin_fmaf(ry, Fy, rx * Fx));
    const float ir2 = ir * ir;
    const float tt = fr * ir2;
    if (RPY) {
        const float ir3 = ir * ir2;
        const float av = __builtin_fmaf(crr, ir3, ir);
        const float bv = tt * __builtin_fmaf(-3.0f * crr, ir3, ir);
        px = __builtin_fmaf(av, Fx, __builtin_fmaf(bv, rx, px));
        py = __builtin_fmaf(av, Fy, __builtin_fmaf(bv, ry, py));
        pz = __builtin_fmaf(av, Fz, __builtin_fmaf(bv, rz, pz));
    } else {
        px = __builtin_fmaf(ir, __builtin_fmaf(tt, rx, Fx), px);
        py = __builtin_fmaf(ir, __builtin_fmaf(tt, ry, Fy), py);
        pz = __builtin_fmaf(ir, __builtin_fmaf(tt, rz, Fz), pz);
    }
}

/* One thread's entry of a source tile: sphere t0 + t of the pack, or
 * padding (far away and force-free, so it contributes exactly zero). */
__device__ __forceinline__ void load_tile_entry(const Dev& d, int t0, int jend, int t, float4& A, float4& B,
                                                float& C) {
    if (t0 + t < jend) {
        A = d.pA[t0 + t];
        B = d.pB[t0 + t];
        C = d.pC[t0 + t].y;
    } else {
        A = make_float4(1.0e15f, 1.0e15f, 1.0e15f, 0.f);
        B = make_float4(0.f, 0.f, 0.f, 0.f);
        C = 0.f;
    }
}

/* append source j to the steric candidate list of target i (i < iend) */
__device__ __noinline__ void add_candidate(const Dev& d, int i, int iend, int j) {
    if (i >= iend) return;
    /* unsigned test: a count outside [0, NBR_CAP) never becomes an index */
    const unsigned k = (unsigned)atomicAdd(&d.nbr_cnt[i], 1);
    if (k < (unsigned)NBR_CAP)
        d.nbr_idx[i * NBR_CAP + (int)k] = j;
    else
        atomicOr(&d.ctl->flag, FLAG_NBR_FULL);
}


/* FP32C pair sum. A work-group of WG threads is WI x WJ waves: WI waves own
 * different target spheres (IPL consecutive spheres per lane), and the WJ
 * waves that share the same targets take interleaved parts of every j-tile.
 * A tile of WG source spheres is staged through LDS once and read as
 * broadcasts.
 *   SPLIT = 1: positions are hi + lo floats, r = (hi_i - hi_j) + (lo_i - lo_j)
 *              (r rounded relative to itself).
 *   SPLIT = 0: positions are single floats, r = x_i - x_j (error ~ eps |x|).
 * Pair math in FP32 with the hardware reciprocal square root. Each wave sums
 * the terms of one tile in FP32 and adds that tile sum to a (hi, lo)
 * accumulator with TwoSum; the WJ waves' accumulators are combined in LDS
 * in a fixed order. The dumbbell's own two spheres are skipped (their terms
 * are in u0, in FP64).
 *   STERIC = 1: every pair closer than rc + skin (r^2 is at hand) is appended
 *              to the target's candidate list for the next stage's steric
 *              forces.
 *   RPY = 1: the pair tensor carries the Rotne-Prager-Yamakawa-Mazur
 *              correction, summed with the Oseen part as
 *              F (ir + c' ir^3) + r t (ir - 3 c' ir^3), c' = 2a^2/3.
 * mode: 0 = mobility apply, 1 = step stage. */
template <int WG, int IPL, int WJ, int SPLIT, int STERIC, int RPY>
__global__ __launch_bounds__(WG) void k_pairs_f32c(Dev d, Epi e, int mode) {
    constexpr int WI = WG / 64 / WJ;
    constexpr int TJ = WG;          /* j per LDS tile */
    constexpr int IB = 64 * WI * IPL;
    /* one LDS area, used in turn by the source tiles and the cross-wave
     * combination (a barrier separates the uses) */
    union Lds {
        struct {
            float4 A[TJ];
            float4 B[TJ];
            float C[TJ];
        } tile;
        float red[WJ > 1 ? WJ : 1][IB][6];
    };
    __shared__ Lds lds;
    float4* sA = lds.tile.A;
    float4* sB = lds.tile.B;
    float* sC = lds.tile.C;
    const Item it = d.items[blockIdx.x];
    if (mode) advance_slots(d, e);
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int wi = wave % WI;
    const int wj = wave / WI;
    const int slot = wi * 64 + lane;          /* target slot inside the block */
    const int ib = it.i0 + slot * IPL;
    const int iend = it.i0 + it.ni;

    float hx[IPL], hy[IPL], hz[IPL], lx[IPL], ly[IPL], lz[IPL];
    float ax[IPL], ay[IPL], az[IPL];  /* running (hi) sums */
    float bx[IPL], by[IPL], bz[IPL];  /* compensation (lo) */
    float px[IPL], py[IPL], pz[IPL];  /* tile partial */
    int dq[IPL];                      /* dumbbell of each target */
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int i = ib + q;
        float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
        if (i < iend) {
            A = d.pA[i];
            B = d.pB[i];
        }
        hx[q] = A.x; hy[q] = A.y; hz[q] = A.z;
        lx[q] = SPLIT ? B.x : 0.f; ly[q] = SPLIT ? B.y : 0.f; lz[q] = SPLIT ? B.z : 0.f;
        ax[q] = ay[q] = az[q] = 0.f;
        bx[q] = by[q] = bz[q] = 0.f;
        px[q] = py[q] = pz[q] = 0.f;
        dq[q] = i >> 1;
    }
    const int dlo = it.i0 & ~1;
    const int dhi = (iend + 1) & ~1;
    const int jend = it.j0 + it.nj;
    const float crr = e.c.crr;

    for (int t0 = it.j0; t0 < jend; t0 += TJ) {
        const int n = min(TJ, jend - t0);
        float4 A, B;
        float C;
        load_tile_entry(d, t0, jend, t, A, B, C);
        __syncthreads();
        sA[t] = A;
        sB[t] = B;
        sC[t] = C;
        __syncthreads();
        const bool diag = (t0 < dhi) && (t0 + n > dlo);
        /* this wave's part of the tile: the n entries in WJ runs of a
         * multiple of 4 (WJ runs of 4 ceil(n / 4WJ) never pass TJ) */
        const int jw = WJ == 1 ? n : (n + 4 * WJ - 1) / (4 * WJ) * 4;
        const int jb = wj * jw;
        const int nw = max(0, min(jw, n - jb));
        if (!diag) {
            const int n4 = (nw + 3) & ~3;
            for (int jj = jb; jj < jb + n4; jj += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float4 Aj = sA[jj + u];
                    const float4 Bj = sB[jj + u];
                    const float Fz = sC[jj + u];
#pragma unroll
                    for (int q = 0; q < IPL; ++q) {
                        float rx, ry, rz;
                        if (SPLIT) {
                            rx = (hx[q] - Aj.x) + (lx[q] - Bj.x);
                            ry = (hy[q] - Aj.y) + (ly[q] - Bj.y);
                            rz = (hz[q] - Aj.z) + (lz[q] - Bj.z);
                        } else {
                            rx = hx[q] - Aj.x;
                            ry = hy[q] - Aj.y;
                            rz = hz[q] - Aj.z;
                        }
                        float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
                        if (STERIC && r2 < d.list_r2) add_candidate(d, ib + q, iend, t0 + jj + u);
                        float ir = __builtin_amdgcn_rsqf(r2);
                        pair_term<RPY>(ir, rx, ry, rz, Aj.w, Bj.w, Fz, crr, px[q], py[q], pz[q]);
                    }
                }
            }
        } else {
            for (int jj = jb; jj < jb + nw; ++jj) {
                const float4 Aj = sA[jj];
                const float4 Bj = sB[jj];
                const float Fz = sC[jj];
                const int dj = (t0 + jj) >> 1;
#pragma unroll
                for (int q = 0; q < IPL; ++q) {
                    float rx, ry, rz;
                    if (SPLIT) {
                        rx = (hx[q] - Aj.x) + (lx[q] - Bj.x);
                        ry = (hy[q] - Aj.y) + (ly[q] - Bj.y);
                        rz = (hz[q] - Aj.z) + (lz[q] - Bj.z);
                    } else {
                        rx = hx[q] - Aj.x;
                        ry = hy[q] - Aj.y;
                        rz = hz[q] - Aj.z;
                    }
                    float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
                    if (STERIC && r2 < d.list_r2 && t0 + jj != ib + q) add_candidate(d, ib + q, iend, t0 + jj);
                    float ir = (dj == dq[q]) ? 0.f : __builtin_amdgcn_rsqf(r2);
                    pair_term<RPY>(ir, rx, ry, rz, Aj.w, Bj.w, Fz, crr, px[q], py[q], pz[q]);
                }
            }
        }
        /* TwoSum of the tile partial into (hi, lo) */
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            two_sum_acc(ax[q], bx[q], px[q]);
            two_sum_acc(ay[q], by[q], py[q]);
            two_sum_acc(az[q], bz[q], pz[q]);
            px[q] = py[q] = pz[q] = 0.f;
        }
    }
    if (WJ > 1) {
        /* combine the WJ waves that share these targets, in wave order */
        __syncthreads(); /* the last tile is no longer read */
        if (wj > 0) {
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                float* r = lds.red[wj][slot * IPL + q];
                r[0] = ax[q]; r[1] = bx[q]; r[2] = ay[q]; r[3] = by[q]; r[4] = az[q]; r[5] = bz[q];
            }
        }
        __syncthreads();
        if (wj == 0) {
#pragma unroll
            for (int w = 1; w < WJ; ++w) {
#pragma unroll
                for (int q = 0; q < IPL; ++q) {
                    const float* r = lds.red[w][slot * IPL + q];
                    two_sum_acc(ax[q], bx[q], r[0]); bx[q] = bx[q] + r[1];
                    two_sum_acc(ay[q], by[q], r[2]); by[q] = by[q] + r[3];
                    two_sum_acc(az[q], bz[q], r[4]); bz[q] = bz[q] + r[5];
                }
            }
        }
    }
    if (wj == 0) {
        const long long base = d.sys_pbase[it.sys] + (long long)it.c * d.ncomp * it.Nb;
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            const int i = ib + q;
            if (i < iend) {
                const int li = i - it.ioff;
                d.part[base + li] = (double)ax[q] + (double)bx[q];
                d.part[base + it.Nb + li] = (double)ay[q] + (double)by[q];
                d.part[base + 2 * it.Nb + li] = (double)az[q] + (double)bz[q];
            }
        }
    }
}

/* ------------------------------------------------------- fused stage */

/* One stage in one kernel. A work-group of NW waves owns FS_I = 16 target
 * spheres of one system and holds all of that system's sources in LDS: lane
 * (wave w, quarter g, target t) sums target t over the sources
 * j = JS m + 4w + g (JS = 4 NW source splits, m = 0, 1, ...) in FP32, with a
 * TwoSum into a (hi, lo) pair every FS_M sources (32 for one system, 64 for
 * an ensemble). The JS partial sums of a target are combined in a fixed order
 * (two shuffles inside the wave, then the NW waves through LDS in a pairwise
 * tree), and wave 0 then does the stage update, next spring forces and next
 * pack of the 8 dumbbells (as the epilogue does, in the rsqrt forms) with no
 * further barrier: a stage needs no partial sums in HBM and no second
 * launch. Only the one term of the
 * JS-source block that holds the work-group's own dumbbells needs the
 * self/partner mask. A single system uses NW = 16 and target blocks in
 * order; an ensemble NW = 4 and a work list of (system, target block),
 * longest system first. */
constexpr int FS_I = 16;

/* One source entry of the fused stage: sphere t0 + t of the pack, or
 * padding (far away and force-free). With single-float positions only
 * A = (x, y, z, Fx) and C = (Fy, Fz) are read, 24 B per source. */
template <int SPLIT>
__device__ __forceinline__ void load_stage_entry(const Dev& d, int t0, int jend, int t, float4& A, float4& B,
                                                 float& Fy, float& Fz) {
    if (t0 + t < jend) {
        A = d.pA[t0 + t];
        if (SPLIT) {
            B = d.pB[t0 + t];
            Fy = B.w;
            Fz = d.pC[t0 + t].y;
        } else {
            const float2 c = d.pC[t0 + t];
            Fy = c.x;
            Fz = c.y;
        }
    } else {
        A = make_float4(1.0e15f, 1.0e15f, 1.0e15f, 0.f);
        B = make_float4(0.f, 0.f, 0.f, 0.f);
        Fy = 0.f;
        Fz = 0.f;
    }
}

template <int SPLIT, int RPY, int NW>
__global__ __launch_bounds__(64 * NW) void k_stage_fused(Dev d, Epi e) {
    constexpr int T = 64 * NW; /* lanes */
    constexpr int JS = 4 * NW; /* source splits per target */
    /* sources per FP32 partial sum before it is folded into (hi, lo) */
    constexpr int FS_M = NW == 16 ? 32 : 64;
    extern __shared__ float4 fs_lds[];
    const int N = d.Ntot;
    const int tid = threadIdx.x;

    /* the work-group's targets [i0, i0 + ni) in the system [off, off + Nb) */
    int i0, ni, off, Nb;
    if (d.nfitems == 0) {
        i0 = blockIdx.x * FS_I;
        off = 0;
        Nb = N;
    } else {
        const Item it = d.fitems[blockIdx.x];
        i0 = it.i0;
        off = it.ioff;
        Nb = it.Nb;
    }
    ni = min(FS_I, off + Nb - i0);
    const int np = (Nb + JS - 1) / JS * JS;
    /* sources: A = (x, y, z, Fx) [np]; with hi/lo B = (lo.x, lo.y, lo.z, Fy)
     * [np] and Fz [np], else (Fy, Fz) [np] */
    float4* sA = fs_lds;
    float4* sB = fs_lds + np;
    float* sC = reinterpret_cast<float*>(fs_lds + 2 * np);
    float2* sF = reinterpret_cast<float2*>(fs_lds + np);
    const long long step = (e.stage == 0) ? d.ctl->slot[0] : d.ctl->slot[1];
    /* inputs of the closing update, loaded first: lane 3t + a owns
     * component a of target i0 + t */
    double u0 = 0.0, xv = 0.0, rv = 0.0;
    if (tid < 3 * ni) {
        const int tt = tid / 3, a = tid - 3 * tt;
        const int o = a * N + i0 + tt;
        u0 = d.U0[o];
        xv = d.X[o];
        if (e.stage > 0) rv = d.R[o];
    }

    const int w = tid >> 6, l = tid & 63, t = l & 15, g = l >> 4;
    const int js = 4 * w + g;
    const int i = i0 + t;
    /* this lane's target position */
    float hx = 0.f, hy = 0.f, hz = 0.f, lx = 0.f, ly = 0.f, lz = 0.f;
    if (t < ni) {
        const float4 A = d.pA[i];
        hx = A.x; hy = A.y; hz = A.z;
        if (SPLIT) {
            const float4 B = d.pB[i];
            lx = B.x; ly = B.y; lz = B.z;
        }
    }

    /* the system's sources into LDS (padding far away and force-free) */
    for (int j = tid; j < np; j += T) {
        float4 A, B;
        float Fy, Fz;
        load_stage_entry<SPLIT>(d, off, off + Nb, j, A, B, Fy, Fz);
        sA[j] = A;
        if (SPLIT) {
            sB[j] = B;
            sC[j] = Fz;
        } else {
            sF[j] = make_float2(Fy, Fz);
        }
    }
    const int di = (i - off) >> 1; /* local dumbbell (off is even) */
    __syncthreads();
    /* after the staging barrier, so that their dependent loads stall only
     * wave 0, whose sums are not the last to finish: the step slots for the
     * next kernel, and for lane q < ni the phase of dumbbell q/2 and the
     * (sin, cos)(omega t) of this stage */
    advance_slots(d, e);
    double st = 0.0, ct = 0.0;
    double2 tp = make_double2(0.0, 0.0);
    if (tid < ni) {
        const long long row = step & (d.ring - 1);
        st = d.tab[row * 8 + 2 * e.stage];
        ct = d.tab[row * 8 + 2 * e.stage + 1];
        tp = d.phitrig[(i0 >> 1) + (tid >> 1)];
    }

    const float crr = e.c.crr;
    float ax = 0.f, ay = 0.f, az = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
    auto term = [&](int j, bool masked, float& px, float& py, float& pz) {
        const float4 Aj = sA[j];
        float Fy, Fz, qx = 0.f, qy = 0.f, qz = 0.f;
        if (SPLIT) {
            const float4 Bj = sB[j];
            qx = Bj.x; qy = Bj.y; qz = Bj.z;
            Fy = Bj.w;
            Fz = sC[j];
        } else {
            const float2 f = sF[j];
            Fy = f.x;
            Fz = f.y;
        }
        float rx, ry, rz;
        if (SPLIT) {
            rx = (hx - Aj.x) + (lx - qx);
            ry = (hy - Aj.y) + (ly - qy);
            rz = (hz - Aj.z) + (lz - qz);
        } else {
            rx = hx - Aj.x;
            ry = hy - Aj.y;
            rz = hz - Aj.z;
        }
        const float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
        float ir = __builtin_amdgcn_rsqf(r2);
        if (masked && (j >> 1) == di) ir = 0.f;
        pair_term<RPY>(ir, rx, ry, rz, Aj.w, Fy, Fz, crr, px, py, pz);
    };
    const int M = np / JS;
    const int ms = (i0 - off) / JS; /* the source block holding this group's dumbbells */
    for (int m0 = 0; m0 < M; m0 += FS_M) {
        const int m1 = min(M, m0 + FS_M);
        float px = 0.f, py = 0.f, pz = 0.f;
        if (ms >= m0 && ms < m1) {
#pragma unroll 4
            for (int m = m0; m < ms; ++m) term(js + JS * m, false, px, py, pz);
            term(js + JS * ms, true, px, py, pz);
#pragma unroll 4
            for (int m = ms + 1; m < m1; ++m) term(js + JS * m, false, px, py, pz);
        } else if (m1 - m0 == FS_M) {
#pragma unroll 4
            for (int m = m0; m < m0 + FS_M; ++m) term(js + JS * m, false, px, py, pz);
        } else {
            for (int m = m0; m < m1; ++m) term(js + JS * m, false, px, py, pz);
        }
        two_sum_acc(ax, bx, px);
        two_sum_acc(ay, by, py);
        two_sum_acc(az, bz, pz);
    }

    /* combine the JS partial sums of each target in a fixed order: the four
     * quarters of a wave by shuffles (both partners get the same sum), then
     * the NW waves through LDS in a pairwise tree */
    auto combine = [](float& hi, float& lo, float oh, float ol) {
        const float s = hi + oh;
        const float bb = s - hi;
        const float err = (hi - (s - bb)) + (oh - bb);
        hi = s;
        lo = (lo + ol) + err;
    };
#pragma unroll
    for (int sh = 16; sh <= 32; sh *= 2) {
        const float oax = __shfl_xor(ax, sh), obx = __shfl_xor(bx, sh);
        const float oay = __shfl_xor(ay, sh), oby = __shfl_xor(by, sh);
        const float oaz = __shfl_xor(az, sh), obz = __shfl_xor(bz, sh);
        combine(ax, bx, oax, obx);
        combine(ay, by, oay, oby);
        combine(az, bz, oaz, obz);
    }
    __syncthreads(); /* the sources are no longer read */
    float* red = reinterpret_cast<float*>(fs_lds);                  /* [NW waves][FS_I][6] */
    double* ys = reinterpret_cast<double*>(fs_lds) + NW * FS_I * 3; /* [FS_I][3] stage positions */
    if (g == 0) {
        float* r = red + (w * FS_I + t) * 6;
        r[0] = ax; r[1] = bx; r[2] = ay; r[3] = by; r[4] = az; r[5] = bz;
    }
    __syncthreads();
    /* wave 0 closes the stage alone */
    if (w != 0) return;
    int bad = 0;
    if (tid < 3 * ni) {
        /* component a of target tt: the waves' sums combined pairwise in a
         * fixed tree (wave w with w + 1, then pairs of pairs, ...), then the
         * stage update */
        const int tt = tid / 3, a = tid - 3 * tt;
        float hs[NW], ls[NW];
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            const float* r = red + (ww * FS_I + tt) * 6 + 2 * a;
            hs[ww] = r[0];
            ls[ww] = r[1];
        }
#pragma unroll
        for (int sp = 1; sp < NW; sp *= 2)
#pragma unroll
            for (int ww = 0; ww < NW; ww += 2 * sp) combine(hs[ww], ls[ww], hs[ww + sp], ls[ww + sp]);
        const int ii = i0 + tt;
        const double k = u0 + e.c.co * ((double)hs[0] + (double)ls[0]);
        bad = !isfinite(k);
        ys[tt * 3 + a] = stage_update(d, e, a * N + ii, ii, a, k, xv, rv, step);
    }
    /* LDS operations of one wave complete in order: the fences only keep
     * the compiler from moving the reads of ys above its writes */
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (__any(bad) && tid == 0) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
    if (tid < ni) {
        /* one lane per sphere: the spring forces of its dumbbell (both lanes
         * of a dumbbell evaluate the same expression, so they agree bit for
         * bit), then its partner term and its part of the next pack */
        const int q = tid >> 1, h = tid & 1;
        double f[2][3];
        spring_forces_rs(e.c, ys + (2 * q) * 3, ys + (2 * q + 1) * 3, tp.x, tp.y, st, ct, f[0], f[1]);
        store_pack_sphere_rs<SPLIT>(d, e.c, i0 + tid, ys + tid * 3, ys + (tid ^ 1) * 3, f[h], f[h ^ 1]);
    }
}

/* Wide form of the fused stage, for ensembles of small systems: a work-group
 * of 4 waves owns FW_I = 64 target spheres of one system, one per lane, and
 * holds all of the system's sources in LDS. Wave w sums, for every target,
 * the sources of its quarter [w Q, (w + 1) Q) of the padded source list
 * (Q = np / 4), each read as an LDS broadcast, in FP32 with a TwoSum into
 * (hi, lo) every FW_M sources. Only the sources that are the work-group's own
 * spheres need the self/partner test. The quarters' sums of a target are
 * combined through LDS as (q0 + q1) + (q2 + q3), and the closing update is
 * the one of k_stage_fused. Per work-group, staging and the closing update
 * cost what they cost for 16 targets, over four times the pair work. */
constexpr int FW_M = 32;

template <int SPLIT, int RPY>
__global__ __launch_bounds__(256) void k_stage_wide(Dev d, Epi e) {
    extern __shared__ float4 fs_lds[];
    const int N = d.Ntot;
    const int tid = threadIdx.x;
    const Item it = d.fitems[blockIdx.x];
    const int i0 = it.i0, off = it.ioff, Nb = it.Nb;
    const int ni = min(FW_I, off + Nb - i0);
    const int np = (Nb + 3) / 4 * 4;
    const int Q = np / 4;
    float4* sA = fs_lds;
    float4* sB = fs_lds + np;
    float* sC = reinterpret_cast<float*>(fs_lds + 2 * np);
    float2* sF = reinterpret_cast<float2*>(fs_lds + np);
    const long long step = (e.stage == 0) ? d.ctl->slot[0] : d.ctl->slot[1];
    /* inputs of the closing update, loaded first: lane 3t + a owns
     * component a of target i0 + t */
    double u0 = 0.0, xv = 0.0, rv = 0.0;
    if (tid < 3 * ni) {
        const int tt = tid / 3, a = tid - 3 * tt;
        const int o = a * N + i0 + tt;
        u0 = d.U0[o];
        xv = d.X[o];
        if (e.stage > 0) rv = d.R[o];
    }
    const int w = tid >> 6, l = tid & 63;
    const int i = i0 + l;
    /* this lane's target position (lanes past the block's end sum for
     * position zero and are not used) */
    float hx = 0.f, hy = 0.f, hz = 0.f, lx = 0.f, ly = 0.f, lz = 0.f;
    if (l < ni) {
        const float4 A = d.pA[i];
        hx = A.x; hy = A.y; hz = A.z;
        if (SPLIT) {
            const float4 B = d.pB[i];
            lx = B.x; ly = B.y; lz = B.z;
        }
    }
    /* the system's sources into LDS (padding far away and force-free) */
    for (int j = tid; j < np; j += 256) {
        float4 A, B;
        float Fy, Fz;
        load_stage_entry<SPLIT>(d, off, off + Nb, j, A, B, Fy, Fz);
        sA[j] = A;
        if (SPLIT) {
            sB[j] = B;
            sC[j] = Fz;
        } else {
            sF[j] = make_float2(Fy, Fz);
        }
    }
    const int di = (i - off) >> 1; /* local dumbbell (off is even) */
    __syncthreads();
    /* as in k_stage_fused: after the staging barrier, for wave 0 only */
    advance_slots(d, e);
    double st = 0.0, ct = 0.0;
    double2 tp = make_double2(0.0, 0.0);
    if (tid < ni) {
        const long long row = step & (d.ring - 1);
        st = d.tab[row * 8 + 2 * e.stage];
        ct = d.tab[row * 8 + 2 * e.stage + 1];
        tp = d.phitrig[(i0 >> 1) + (tid >> 1)];
    }

    const float crr = e.c.crr;
    float ax = 0.f, ay = 0.f, az = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
    auto term = [&](int j, bool masked, float& px, float& py, float& pz) {
        const float4 Aj = sA[j];
        float Fy, Fz, qx = 0.f, qy = 0.f, qz = 0.f;
        if (SPLIT) {
            const float4 Bj = sB[j];
            qx = Bj.x; qy = Bj.y; qz = Bj.z;
            Fy = Bj.w;
            Fz = sC[j];
        } else {
            const float2 f = sF[j];
            Fy = f.x;
            Fz = f.y;
        }
        float rx, ry, rz;
        if (SPLIT) {
            rx = (hx - Aj.x) + (lx - qx);
            ry = (hy - Aj.y) + (ly - qy);
            rz = (hz - Aj.z) + (lz - qz);
        } else {
            rx = hx - Aj.x;
            ry = hy - Aj.y;
            rz = hz - Aj.z;
        }
        const float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
        float ir = __builtin_amdgcn_rsqf(r2);
        if (masked && (j >> 1) == di) ir = 0.f;
        pair_term<RPY>(ir, rx, ry, rz, Aj.w, Fy, Fz, crr, px, py, pz);
    };
    /* this wave's quarter of the sources, and the part of it that holds the
     * work-group's own spheres (local [i0 - off, i0 - off + ni)) */
    const int j0 = w * Q, j1 = j0 + Q;
    const int jm0 = max(j0, i0 - off), jm1 = min(j1, i0 - off + ni);
    for (int c0 = j0; c0 < j1; c0 += FW_M) {
        const int c1 = min(j1, c0 + FW_M);
        float px = 0.f, py = 0.f, pz = 0.f;
        if (c0 < jm1 && c1 > jm0) {
            for (int j = c0; j < c1; ++j) term(j, true, px, py, pz);
        } else if (c1 - c0 == FW_M) {
#pragma unroll 4
            for (int j = c0; j < c0 + FW_M; ++j) term(j, false, px, py, pz);
        } else {
            for (int j = c0; j < c1; ++j) term(j, false, px, py, pz);
        }
        two_sum_acc(ax, bx, px);
        two_sum_acc(ay, by, py);
        two_sum_acc(az, bz, pz);
    }

    auto combine = [](float& hi, float& lo, float oh, float ol) {
        const float s = hi + oh;
        const float bb = s - hi;
        const float err = (hi - (s - bb)) + (oh - bb);
        hi = s;
        lo = (lo + ol) + err;
    };
    __syncthreads(); /* the sources are no longer read */
    float* red = reinterpret_cast<float*>(fs_lds);                   /* [4 waves][FW_I][6] */
    double* ys = reinterpret_cast<double*>(fs_lds) + 4 * FW_I * 3;   /* [FW_I][3] stage positions */
    int* badf = reinterpret_cast<int*>(ys + FW_I * 3);
    {
        float* r = red + (w * FW_I + l) * 6;
        r[0] = ax; r[1] = bx; r[2] = ay; r[3] = by; r[4] = az; r[5] = bz;
    }
    if (tid == 0) *badf = 0;
    __syncthreads();
    if (tid < 3 * ni) {
        const int tt = tid / 3, a = tid - 3 * tt;
        float hs[4], ls[4];
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
            const float* r = red + (ww * FW_I + tt) * 6 + 2 * a;
            hs[ww] = r[0];
            ls[ww] = r[1];
        }
        combine(hs[0], ls[0], hs[1], ls[1]);
        combine(hs[2], ls[2], hs[3], ls[3]);
        combine(hs[0], ls[0], hs[2], ls[2]);
        const int ii = i0 + tt;
        const double k = u0 + e.c.co * ((double)hs[0] + (double)ls[0]);
        if (!isfinite(k)) *badf = 1;
        ys[tt * 3 + a] = stage_update(d, e, a * N + ii, ii, a, k, xv, rv, step);
    }
    __syncthreads();
    if (tid == 0 && *badf) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
    if (tid < ni) {
        /* one lane per sphere, as in k_stage_fused */
        const int q = tid >> 1, h = tid & 1;
        double f[2][3];
        spring_forces_rs(e.c, ys + (2 * q) * 3, ys + (2 * q + 1) * 3, tp.x, tp.y, st, ct, f[0], f[1]);
        store_pack_sphere_rs<SPLIT>(d, e.c, i0 + tid, ys + tid * 3, ys + (tid ^ 1) * 3, f[h], f[h ^ 1]);
    }
}

/* Streamed form of the fused stage (ad_launch.fused = 3). The work-group of
 * NW waves owns TI target spheres. TI = 4, 8 or 16 (stream_targets) keeps
 * about one work-group per compute unit: at N = 4096, TI = 8 puts two
 * work-groups on a compute unit and measured 22 % slower, since every
 * work-group reads every source; at N = 2048, TI = 16 leaves half the compute
 * units idle and measured 18 % slower. NW = 16, or 8 with 4 targets
 * (stream_waves): with 8 waves N = 512 ran 16 % faster and N = 1024 9 %, while
 * N = 4096 with 16 targets ran 10 % slower. Each of its source splits
 * (wave w, lane group g of TI lanes) owns a contiguous range of Q sources
 * (Q a multiple of TI). A wave streams its ranges through a double-buffered LDS
 * slot of its own, TI sources per split at a time, one entry per lane: the
 * loads of the chunk after next are in flight while the current chunk is
 * summed (two register sets; 0.5 % off a 4096-sphere step, 1.3 % at 8192), no
 * work-group barrier separates loading from summing, and no system is too
 * large for LDS. Lane (w, g, t) sums target t over its split's range in
 * ascending order, folding into (hi, lo) every 32 sources. LDS ops of one
 * wave complete in order, so the slot needs no barrier: a chunk is written
 * after the wave's reads of the chunk it replaces and read after its own
 * writes. (Interleaving the groups' entries within a slot measured slower.)
 * The partial sums are combined in k_stage_fused's order, through an LDS
 * area beside the slots, so one work-group barrier precedes the closing
 * update; wave 0 then does it alone (stage update, spring forces and pack,
 * in the rsqrt forms) with no further barrier.
 * BAL: with one work-group per compute unit, the waves of a SIMD keep pace:
 * a wave lowers its issue priority one step per quarter of its chunks, so
 * the SIMD issues from the waves that are behind. Under the default oldest-
 * first choice the first waves finish early and the last run with fewer
 * waves to hide their latencies; kept in step, all four waves issue until
 * the end (N = 4096: 7 % off the step). With two work-groups per compute
 * unit the early finishers' closing update overlaps the other work-group's
 * sums instead, and keeping pace was 6 % slower (N = 8192), as it was with
 * fewer chunks per lane (1-3 % at N = 512 and 2048). */
template <int SPLIT, int RPY, int TI, int NW, int BAL>
__device__ __forceinline__ void stage_stream(const Dev& d, const Epi& e) {
    constexpr int G = 64 / TI;    /* lane groups (splits) per wave */
    constexpr int JS = NW * G;    /* source splits */
    constexpr int FOLD = 32 / TI; /* chunks per (hi, lo) fold */
    extern __shared__ float4 fs_lds[];
    const int N = d.Ntot;
    const int tid = threadIdx.x;
    int i0, off, Nb;
    if (d.nfitems == 0) {
        i0 = blockIdx.x * TI;
        off = 0;
        Nb = N;
    } else {
        const Item it = d.fitems[blockIdx.x];
        i0 = it.i0;
        off = it.ioff;
        Nb = it.Nb;
    }
    const int ni = min(TI, off + Nb - i0);
    const int Q = (Nb + JS * TI - 1) / (JS * TI) * TI; /* sources per split */
    const int K = Q / TI;                              /* chunks per split */
    /* per wave and buffer 64 entries: A = (x, y, z, Fx); with hi/lo
     * B = (lo.xyz, Fy) and Fz, else (Fy, Fz) */
    float4* sA = fs_lds;
    float4* sB = fs_lds + NW * 128;
    float* sC = reinterpret_cast<float*>(fs_lds + 2 * NW * 128);
    float2* sF = reinterpret_cast<float2*>(fs_lds + NW * 128);
    const long long step = (e.stage == 0) ? d.ctl->slot[0] : d.ctl->slot[1];
    /* inputs of the closing update, loaded first */
    double u0 = 0.0, xv = 0.0, rv = 0.0;
    if (tid < 3 * ni) {
        const int tt = tid / 3, a = tid - 3 * tt;
        const int o = a * N + i0 + tt;
        u0 = d.U0[o];
        xv = d.X[o];
        if (e.stage > 0) rv = d.R[o];
    }
    const int w = tid >> 6, l = tid & 63, t = l % TI, g = l / TI;
    const int sp = G * w + g; /* this lane's source split */
    const int i = i0 + t;
    float hx = 0.f, hy = 0.f, hz = 0.f, lx = 0.f, ly = 0.f, lz = 0.f;
    if (t < ni) {
        const float4 A = d.pA[i];
        hx = A.x; hy = A.y; hz = A.z;
        if (SPLIT) {
            const float4 B = d.pB[i];
            lx = B.x; ly = B.y; lz = B.z;
        }
    }
    const int di = (i - off) >> 1;
    /* the chunk holding the work-group's own spheres: split so, chunk ko */
    const int so = (i0 - off) / Q, ko = ((i0 - off) - so * Q) / TI;
    const bool own_wave = so / G == w;

    /* two register sets: chunk k + 2 is loaded while chunk k is summed */
    float4 eA0, eB0, eA1, eB1;
    float eFy0, eFz0, eFy1, eFz1;
    auto fetch = [&](int k, auto R) {
        if constexpr (decltype(R)::value == 0)
            load_stage_entry<SPLIT>(d, off, off + Nb, sp * Q + k * TI + t, eA0, eB0, eFy0, eFz0);
        else
            load_stage_entry<SPLIT>(d, off, off + Nb, sp * Q + k * TI + t, eA1, eB1, eFy1, eFz1);
    };
    auto put = [&](int buf, auto R) {
        constexpr int r = decltype(R)::value;
        const int x = (w * 2 + buf) * 64 + g * TI + t;
        sA[x] = r ? eA1 : eA0;
        if (SPLIT) {
            sB[x] = r ? eB1 : eB0;
            sC[x] = r ? eFz1 : eFz0;
        } else {
            sF[x] = r ? make_float2(eFy1, eFz1) : make_float2(eFy0, eFz0);
        }
    };
    fetch(0, std::integral_constant<int, 0>{});
    put(0, std::integral_constant<int, 0>{});
    if (K > 1) fetch(1, std::integral_constant<int, 1>{});
    /* wave 0 only: the step slots and this stage's (sin, cos)(omega t) and
     * phases, whose dependent loads then stall a wave that is not the last
     * to finish its sums */
    advance_slots(d, e);
    double st = 0.0, ct = 0.0;
    double2 tp = make_double2(0.0, 0.0);
    if (tid < ni) {
        const long long row = step & (d.ring - 1);
        st = d.tab[row * 8 + 2 * e.stage];
        ct = d.tab[row * 8 + 2 * e.stage + 1];
        tp = d.phitrig[(i0 >> 1) + (tid >> 1)];
    }

    const float crr = e.c.crr;
    float ax = 0.f, ay = 0.f, az = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
    auto term = [&](int x, int j, bool masked, float& px, float& py, float& pz) {
        const float4 Aj = sA[x];
        float Fy, Fz, qx = 0.f, qy = 0.f, qz = 0.f;
        if (SPLIT) {
            const float4 Bj = sB[x];
            qx = Bj.x; qy = Bj.y; qz = Bj.z;
            Fy = Bj.w;
            Fz = sC[x];
        } else {
            const float2 f = sF[x];
            Fy = f.x;
            Fz = f.y;
        }
        float rx, ry, rz;
        if (SPLIT) {
            rx = (hx - Aj.x) + (lx - qx);
            ry = (hy - Aj.y) + (ly - qy);
            rz = (hz - Aj.z) + (lz - qz);
        } else {
            rx = hx - Aj.x;
            ry = hy - Aj.y;
            rz = hz - Aj.z;
        }
        const float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
        float ir = __builtin_amdgcn_rsqf(r2);
        if (masked && (j >> 1) == di) ir = 0.f;
        pair_term<RPY>(ir, rx, ry, rz, Aj.w, Fy, Fz, crr, px, py, pz);
    };
    float px = 0.f, py = 0.f, pz = 0.f;
    auto chunk = [&](int k, auto R) {
        constexpr int r = decltype(R)::value; /* = k & 1, the buffer and the set of chunk k */
        if (BAL) {
            const int lvl = (4 * k) / K;
            if (lvl == 0) __builtin_amdgcn_s_setprio(3);
            else if (lvl == 1) __builtin_amdgcn_s_setprio(2);
            else if (lvl == 2) __builtin_amdgcn_s_setprio(1);
            else __builtin_amdgcn_s_setprio(0);
        }
        if (k + 2 < K) fetch(k + 2, R);
        const int x0 = (w * 2 + r) * 64 + g * TI;
        const int j0 = sp * Q + k * TI;
        if (own_wave && k == ko) {
            for (int v = 0; v < TI; ++v) term(x0 + v, j0 + v, true, px, py, pz);
        } else {
#pragma unroll
            for (int v = 0; v < TI; ++v) term(x0 + v, j0 + v, false, px, py, pz);
        }
        if ((k + 1) % FOLD == 0 || k + 1 == K) {
            two_sum_acc(ax, bx, px);
            two_sum_acc(ay, by, py);
            two_sum_acc(az, bz, pz);
            px = py = pz = 0.f;
        }
        if (k + 1 < K) put(1 - r, std::integral_constant<int, 1 - r>{});
    };
    for (int k = 0; k < K; k += 2) {
        chunk(k, std::integral_constant<int, 0>{});
        if (k + 1 < K) chunk(k + 1, std::integral_constant<int, 1>{});
    }

    /* combine the partial sums of each target as k_stage_fused does: the G
     * groups of a wave by shuffles, then the waves through LDS in a tree */
    auto combine = [](float& hi, float& lo, float oh, float ol) {
        const float s = hi + oh;
        const float bb = s - hi;
        const float err = (hi - (s - bb)) + (oh - bb);
        hi = s;
        lo = (lo + ol) + err;
    };
#pragma unroll
    for (int sh = TI; sh < 64; sh *= 2) {
        const float oax = __shfl_xor(ax, sh), obx = __shfl_xor(bx, sh);
        const float oay = __shfl_xor(ay, sh), oby = __shfl_xor(by, sh);
        const float oaz = __shfl_xor(az, sh), obz = __shfl_xor(bz, sh);
        combine(ax, bx, oax, obx);
        combine(ay, by, oay, oby);
        combine(az, bz, oaz, obz);
    }
    /* the combination area lies beside the source slots, so no barrier
     * waits for the slowest wave's last reads before it is written */
    float* red = reinterpret_cast<float*>(reinterpret_cast<char*>(fs_lds) + NW * 128 * (SPLIT ? 36 : 24));
    double* ys = reinterpret_cast<double*>(red + NW * TI * 6); /* [TI][3] stage positions */
    if (g == 0) {
        float* r = red + (w * TI + t) * 6;
        r[0] = ax; r[1] = bx; r[2] = ay; r[3] = by; r[4] = az; r[5] = bz;
    }
    __syncthreads();
    /* wave 0 closes the stage alone */
    if (w != 0) return;
    if (BAL) __builtin_amdgcn_s_setprio(3);
    int bad = 0;
    if (tid < 3 * ni) {
        const int tt = tid / 3, a = tid - 3 * tt;
        float hs[NW], ls[NW];
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            const float* r = red + (ww * TI + tt) * 6 + 2 * a;
            hs[ww] = r[0];
            ls[ww] = r[1];
        }
#pragma unroll
        for (int st2 = 1; st2 < NW; st2 *= 2)
#pragma unroll
            for (int ww = 0; ww < NW; ww += 2 * st2) combine(hs[ww], ls[ww], hs[ww + st2], ls[ww + st2]);
        const int ii = i0 + tt;
        const double k = u0 + e.c.co * ((double)hs[0] + (double)ls[0]);
        bad = !isfinite(k);
        ys[tt * 3 + a] = stage_update(d, e, a * N + ii, ii, a, k, xv, rv, step);
    }
    /* LDS operations of one wave complete in order: the fences only keep
     * the compiler from moving the reads of ys above its writes */
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (__any(bad) && tid == 0) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
    if (tid < ni) {
        const int q = tid >> 1, h = tid & 1;
        double f[2][3];
        spring_forces_rs(e.c, ys + (2 * q) * 3, ys + (2 * q + 1) * 3, tp.x, tp.y, st, ct, f[0], f[1]);
        store_pack_sphere_rs<SPLIT>(d, e.c, i0 + tid, ys + tid * 3, ys + (tid ^ 1) * 3, f[h], f[h ^ 1]);
    }
}

template <int SPLIT, int RPY, int TI, int NW>
__global__ __launch_bounds__(64 * NW) void k_stage_stream(Dev d, Epi e) {
    stage_stream<SPLIT, RPY, TI, NW, TI == 16 && NW == 16>(d, e);
}

/* The same with registers capped for 8 waves per SIMD (63 VGPRs), so that two
 * 16-wave work-groups share a compute unit: for launches of more than 256
 * work-groups (N = 8192: 4 % faster per step; with one work-group per compute
 * unit, N = 4096, the cap cost 5 %). */
template <int SPLIT, int RPY, int TI, int NW>
__global__ __launch_bounds__(64 * NW, 8) void k_stage_stream_x2(Dev d, Epi e) {
    stage_stream<SPLIT, RPY, TI, NW, 0>(d, e);
}

/* FP64 streamed form of the fused stage (AD_FP64_TILED with
 * ad_launch.fused = 3): k_stage_stream's work-group shape, streaming and
 * combination order in FP64 arithmetic, for a like-for-like comparison with
 * the FP32C form. The pair term uses v_rsq_f64 refined by one Newton step
 * and FMAs (a relative error of a few ulp, not the IEEE sqrt and divisions
 * of the plain sum); the partial sums are plain FP64 sums. As in the other
 * FP64 forms, the pair sum includes the dumbbell partner and only the self
 * term is masked, u0 is the self term alone, and the pack is the FP64 one
 * (3 double2 per sphere). */
template <int RPY>
__device__ __forceinline__ void pair_term64(double ir, double rx, double ry, double rz, double Fx, double Fy,
                                            double Fz, double crr, double& px, double& py, double& pz) {
    const double fr = __builtin_fma(rz, Fz, __builtin_fma(ry, Fy, rx * Fx));
    const double ir2 = ir * ir;
    const double tt = fr * ir2;
    if (RPY) {
        const double ir3 = ir * ir2;
        const double av = __builtin_fma(crr, ir3, ir);
        const double bv = tt * __builtin_fma(-3.0 * crr, ir3, ir);
        px = __builtin_fma(av, Fx, __builtin_fma(bv, rx, px));
        py = __builtin_fma(av, Fy, __builtin_fma(bv, ry, py));
        pz = __builtin_fma(av, Fz, __builtin_fma(bv, rz, pz));
    } else {
        px = __builtin_fma(ir, __builtin_fma(tt, rx, Fx), px);
        py = __builtin_fma(ir, __builtin_fma(tt, ry, Fy), py);
        pz = __builtin_fma(ir, __builtin_fma(tt, rz, Fz), pz);
    }
}

/* 1/sqrt(r2) from v_rsq_f64 and one Newton step y (1 + (1 - r2 y^2) / 2) */
__device__ __forceinline__ double rsqrt64_nr(double r2) {
    const double y = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2 * y, y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
}

template <int RPY, int TI>
__global__ __launch_bounds__(1024) void k_stage_stream64(Dev d, Epi e) {
    constexpr int NW = 16;
    constexpr int G = 64 / TI;  /* lane groups (splits) per wave */
    constexpr int JS = NW * G;  /* source splits */
    extern __shared__ double4 fs64_lds[];
    const int N = d.Ntot;
    const int tid = threadIdx.x;
    int i0, off, Nb;
    if (d.nfitems == 0) {
        i0 = blockIdx.x * TI;
        off = 0;
        Nb = N;
    } else {
        const Item it = d.fitems[blockIdx.x];
        i0 = it.i0;
        off = it.ioff;
        Nb = it.Nb;
    }
    const int ni = min(TI, off + Nb - i0);
    const int Q = (Nb + JS * TI - 1) / (JS * TI) * TI; /* sources per split */
    const int K = Q / TI;                              /* chunks per split */
    /* per wave and buffer 64 entries: A = (x, y, z, Fx), F = (Fy, Fz) */
    double4* sA = fs64_lds;
    double2* sF = reinterpret_cast<double2*>(fs64_lds + NW * 128);
    const long long step = (e.stage == 0) ? d.ctl->slot[0] : d.ctl->slot[1];
    double u0 = 0.0, xv = 0.0, rv = 0.0;
    if (tid < 3 * ni) {
        const int tt = tid / 3, a = tid - 3 * tt;
        const int o = a * N + i0 + tt;
        u0 = d.U0[o];
        xv = d.X[o];
        if (e.stage > 0) rv = d.R[o];
    }
    const int w = tid >> 6, l = tid & 63, t = l % TI, g = l / TI;
    const int sp = G * w + g;
    const int i = i0 + t;
    double hx = 0.0, hy = 0.0, hz = 0.0;
    if (t < ni) {
        const double2 a0 = d.pD[3 * i], a1 = d.pD[3 * i + 1];
        hx = a0.x; hy = a0.y; hz = a1.x;
    }
    const int so = (i0 - off) / Q, ko = ((i0 - off) - so * Q) / TI;
    const bool own_wave = so / G == w;

    double4 eA;
    double2 eF;
    auto fetch = [&](int k) {
        const int j = sp * Q + k * TI + t;
        if (off + j < off + Nb) {
            const double2 a0 = d.pD[3 * (off + j)], a1 = d.pD[3 * (off + j) + 1], a2 = d.pD[3 * (off + j) + 2];
            eA = make_double4(a0.x, a0.y, a1.x, a1.y);
            eF = a2;
        } else {
            eA = make_double4(1.0e15, 1.0e15, 1.0e15, 0.0);
            eF = make_double2(0.0, 0.0);
        }
    };
    auto put = [&](int buf) {
        const int x = (w * 2 + buf) * 64 + g * TI + t;
        sA[x] = eA;
        sF[x] = eF;
    };
    fetch(0);
    put(0);
    advance_slots(d, e);
    double st = 0.0, ct = 0.0;
    double2 tp = make_double2(0.0, 0.0);
    if (tid < ni) {
        const long long row = step & (d.ring - 1);
        st = d.tab[row * 8 + 2 * e.stage];
        ct = d.tab[row * 8 + 2 * e.stage + 1];
        tp = d.phitrig[(i0 >> 1) + (tid >> 1)];
    }

    const double crr = e.c.crr64;
    double px = 0.0, py = 0.0, pz = 0.0;
    auto term = [&](int x, int j, bool masked) {
        const double4 Aj = sA[x];
        const double2 Fj = sF[x];
        const double rx = hx - Aj.x, ry = hy - Aj.y, rz = hz - Aj.z;
        const double r2 = __builtin_fma(rz, rz, __builtin_fma(ry, ry, rx * rx));
        double ir = rsqrt64_nr(r2);
        if (masked && j == i - off) ir = 0.0;
        pair_term64<RPY>(ir, rx, ry, rz, Aj.w, Fj.x, Fj.y, crr, px, py, pz);
    };
    for (int k = 0; k < K; ++k) {
        const int buf = k & 1;
        if (TI == 16) {
            /* the waves of a SIMD keep pace, as in k_stage_stream's
             * one-work-group-per-unit instance (one 16-wave work-group per
             * compute unit fits at this kernel's register count) */
            const int lvl = (4 * k) / K;
            if (lvl == 0) __builtin_amdgcn_s_setprio(3);
            else if (lvl == 1) __builtin_amdgcn_s_setprio(2);
            else if (lvl == 2) __builtin_amdgcn_s_setprio(1);
            else __builtin_amdgcn_s_setprio(0);
        }
        if (k + 1 < K) fetch(k + 1);
        const int x0 = (w * 2 + buf) * 64 + g * TI;
        const int j0 = sp * Q + k * TI;
        if (own_wave && k == ko) {
            for (int v = 0; v < TI; ++v) term(x0 + v, j0 + v, true);
        } else {
#pragma unroll
            for (int v = 0; v < TI; ++v) term(x0 + v, j0 + v, false);
        }
        if (k + 1 < K) put(buf ^ 1);
    }
    /* the G groups of a wave by shuffles, then the waves through LDS in a
     * pairwise tree: a fixed order */
#pragma unroll
    for (int sh = TI; sh < 64; sh *= 2) {
        px = px + __shfl_xor(px, sh);
        py = py + __shfl_xor(py, sh);
        pz = pz + __shfl_xor(pz, sh);
    }
    double* red = reinterpret_cast<double*>(fs64_lds + NW * 128 + NW * 128 / 2); /* [NW][TI][3] */
    double* ys = red + NW * TI * 3;                                              /* [TI][3] */
    if (g == 0) {
        double* r = red + (w * TI + t) * 3;
        r[0] = px; r[1] = py; r[2] = pz;
    }
    __syncthreads();
    if (w != 0) return;
    if (TI == 16) __builtin_amdgcn_s_setprio(3);
    int bad = 0;
    if (tid < 3 * ni) {
        const int tt = tid / 3, a = tid - 3 * tt;
        double hs[NW];
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) hs[ww] = red[(ww * TI + tt) * 3 + a];
#pragma unroll
        for (int st2 = 1; st2 < NW; st2 *= 2)
#pragma unroll
            for (int ww = 0; ww < NW; ww += 2 * st2) hs[ww] = hs[ww] + hs[ww + st2];
        const int ii = i0 + tt;
        const double k = u0 + e.c.co * hs[0];
        bad = !isfinite(k);
        ys[tt * 3 + a] = stage_update(d, e, a * N + ii, ii, a, k, xv, rv, step);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (__any(bad) && tid == 0) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
    if (tid < ni) {
        const int q = tid >> 1, h = tid & 1;
        double f[2][3];
        spring_forces_rs(e.c, ys + (2 * q) * 3, ys + (2 * q + 1) * 3, tp.x, tp.y, st, ct, f[0], f[1]);
        const double* y = ys + tid * 3;
        const int ii = i0 + tid;
        for (int a = 0; a < 3; ++a) d.U0[a * N + ii] = e.c.cs * f[h][a];
        d.pD2[3 * ii + 0] = make_double2(y[0], y[1]);
        d.pD2[3 * ii + 1] = make_double2(y[2], f[h][0]);
        d.pD2[3 * ii + 2] = make_double2(f[h][1], f[h][2]);
    }
}

/* FP64: the sum in ascending j with the plain operation order
 *   r2 = (rx*rx + ry*ry) + rz*rz; ir = 1/sqrt(r2); fr = (rx*Fx + ry*Fy) + rz*Fz;
 *   t = fr/r2; acc = acc + ir*(F + t*r)
 * over every j != i of the chunk (partner included). A coincident pair is
 * skipped and raises the flag. With one chunk per system this is the
 * sequential FP64 sum exactly (AD_FP64 runs k_pairs_f64w, which gives the
 * same bits); AD_FP64_TILED runs several chunks. With RPY the correction
 * (F - 3 t r) ir/r2 is summed in a second accumulator. */
template <int WG, int IPL, int RPY>
__global__ __launch_bounds__(WG) void k_pairs_f64(Dev d, Epi e, int mode) {
    __shared__ double2 sD[3][WG];
    const Item it = d.items[blockIdx.x];
    if (mode) advance_slots(d, e);
    const int t = threadIdx.x;
    const int ib = it.i0 + t * IPL;
    const int iend = it.i0 + it.ni;
    double xi[IPL], yi[IPL], zi[IPL], ax[IPL], ay[IPL], az[IPL], bx[IPL], by[IPL], bz[IPL];
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int i = ib + q;
        double2 p0 = make_double2(0.0, 0.0), p1 = p0;
        if (i < iend) {
            p0 = d.pD[3 * i];
            p1 = d.pD[3 * i + 1];
        }
        xi[q] = p0.x; yi[q] = p0.y; zi[q] = p1.x;
        ax[q] = ay[q] = az[q] = 0.0;
        bx[q] = by[q] = bz[q] = 0.0;
    }
    int bad = 0;
    const int jend = it.j0 + it.nj;
    for (int t0 = it.j0; t0 < jend; t0 += WG) {
        const int n = min(WG, jend - t0);
        double2 a0, a1, a2;
        if (t < n) {
            a0 = d.pD[3 * (t0 + t)];
            a1 = d.pD[3 * (t0 + t) + 1];
            a2 = d.pD[3 * (t0 + t) + 2];
        } else {
            a0 = make_double2(1.0e300, 1.0e300);
            a1 = make_double2(1.0e300, 0.0);
            a2 = make_double2(0.0, 0.0);
        }
        __syncthreads();
        sD[0][t] = a0;
        sD[1][t] = a1;
        sD[2][t] = a2;
        __syncthreads();
        /* four sources at a time: their terms' square roots and divisions
         * overlap, the additions stay in ascending j (6 % faster than one at
         * a time, 8 at a time 2 %) */
#pragma unroll 4
        for (int jj = 0; jj < n; ++jj) {
            const double2 b0 = sD[0][jj], b1 = sD[1][jj], b2 = sD[2][jj];
            const double Fx = b1.y, Fy = b2.x, Fz = b2.y;
            const int j = t0 + jj;
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                double rx = xi[q] - b0.x;
                double ry = yi[q] - b0.y;
                double rz = zi[q] - b1.x;
                double r2 = (rx * rx + ry * ry) + rz * rz;
                bool self = (j == ib + q);
                bool skip = self || (r2 == 0.0);
                bad |= (!self && r2 == 0.0);
                double r2s = skip ? 1.0 : r2;
                double ir = 1.0 / sqrt(r2s);
                double fr = (rx * Fx + ry * Fy) + rz * Fz;
                double tt = fr / r2s;
                double gx = ir * (Fx + tt * rx);
                double gy = ir * (Fy + tt * ry);
                double gz = ir * (Fz + tt * rz);
                ax[q] = skip ? ax[q] : ax[q] + gx;
                ay[q] = skip ? ay[q] : ay[q] + gy;
                az[q] = skip ? az[q] : az[q] + gz;
                if (RPY) {
                    const double ir3 = ir / r2s;
                    const double t3 = 3.0 * tt;
                    const double hx = ir3 * (Fx - t3 * rx);
                    const double hy = ir3 * (Fy - t3 * ry);
                    const double hz = ir3 * (Fz - t3 * rz);
                    bx[q] = skip ? bx[q] : bx[q] + hx;
                    by[q] = skip ? by[q] : by[q] + hy;
                    bz[q] = skip ? bz[q] : bz[q] + hz;
                }
            }
        }
    }
    const long long base = d.sys_pbase[it.sys] + (long long)it.c * d.ncomp * it.Nb;
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int i = ib + q;
        if (i < iend) {
            const int li = i - it.ioff;
            d.part[base + li] = ax[q];
            d.part[base + it.Nb + li] = ay[q];
            d.part[base + 2 * it.Nb + li] = az[q];
            if (RPY) {
                d.part[base + 3 * it.Nb + li] = bx[q];
                d.part[base + 4 * it.Nb + li] = by[q];
                d.part[base + 5 * it.Nb + li] = bz[q];
            }
            if (bad) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
        }
    }
}

/* Correctly rounded FP64 square root and division in their short forms.
 * The compiler's forms of sqrt(x) and a / b scale the operands' exponents
 * where an intermediate could leave the normal range and fix up special
 * operands (zero, infinity, NaN) afterwards; between those steps they are
 * exactly these instruction sequences (the square root: v_rsq_f64 refined
 * by Newton steps on g = sqrt(x) and h = 1 / (2 sqrt(x)); the division:
 * v_rcp_f64 refined twice, then the quotient corrected once by its
 * residual). For operands where no scaling or fixup applies they give the
 * same bits, which f64_plain_range guarantees with a wide margin: every
 * operand in [2^-400, 2^400], so that no intermediate gets near the ends of
 * the exponent range. */
__device__ __forceinline__ bool f64_plain_range(double x) { return x >= 0x1p-400 && x <= 0x1p400; }
__device__ __forceinline__ double sqrt_plain(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = y * 0.5;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, x);
    return __builtin_fma(d, h, g);
}
__device__ __forceinline__ double div_plain(double a, double b) {
    double y = __builtin_amdgcn_rcp(b);
    double e = __builtin_fma(-b, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-b, y, 1.0);
    y = __builtin_fma(y, e, y);
    const double q = a * y;
    const double r = __builtin_fma(-b, q, a);
    return __builtin_fma(r, y, q);
}

/* Work-group barrier that orders LDS only: vector-memory loads in flight
 * (the step table's next row, the next chunk's sources) are not waited for. */
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

/* AD_FP64 in one kernel, with producer and consumer waves: a work-group owns
 * TW targets of one system. Its NP producer waves form the pair terms of the
 * system's sources in chunks of CW (64 or 128; a lane forms the terms of
 * sources l, l + 64, ... for the TW targets), into LDS rows (component x TW +
 * target) by columns (the chunk's sources); its consumer wave adds them,
 * lane r row r, to a running sum in ascending j. Chunks go in rounds of NP,
 * one per producer, through two sets of buffers: the producers form round
 * m + 1 while the consumer adds round m, and one LDS barrier ends a round
 * (one producer, F64W_NP, measured fastest).
 * The terms are the plain sum's expressions and the additions its sequence,
 * so the result is bitwise k_pairs_f64's with one chunk per system. The
 * self term, a coincident pair (which raises the flag) and the padding past
 * the system's last source are stored as +0.0 and added like the others: a
 * sum that starts at +0.0 is never -0.0 in round-to-nearest, so adding +0.0
 * changes no bit of it. The consumer's lanes past the last row repeat its
 * reads and additions (the same LDS addresses, served once). */
template <int TW, int NP, int CW, int RPY>
__global__ __launch_bounds__(64 * (NP + 1)) void k_pairs_f64w(Dev d, Epi e, int mode) {
    constexpr int NC = RPY ? 6 : 3;
    constexpr int ROWS = NC * TW;
    constexpr int RS = CW + 1;          /* LDS row stride in doubles: odd, so the rows' reads of one
                                           column fall in different banks */
    constexpr int BUF = ROWS * RS; /* doubles per chunk buffer */
    extern __shared__ double w_lds[];   /* [2 sets][NP chunks][ROWS][RS] */
    const Item it = d.fitems[blockIdx.x];
    if (mode) advance_slots(d, e);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    const int Nb = it.Nb, off = it.ioff;
    const int nch = (Nb + CW - 1) / CW;
    const int M = (nch + NP - 1) / NP; /* rounds */
    if (w == 0) {
        /* the consumer */
        const int r = l < ROWS ? l : ROWS - 1;
        double acc = 0.0;
        lds_barrier();
        for (int m = 0; m < M; ++m) {
            const double* S = w_lds + (m & 1) * NP * BUF + r * RS;
            for (int p = 0; p < NP && m * NP + p < nch; ++p) {
                const double* Ta = S + p * BUF;
#pragma unroll
                for (int u = 0; u < CW; ++u) acc = acc + Ta[u];
            }
            lds_barrier();
        }
        if (l < ROWS) {
            const int a = l / TW, q = l - a * TW;
            if (q < it.ni) d.part[d.sys_pbase[it.sys] + (long long)a * Nb + (it.i0 + q - off)] = acc;
        }
        return;
    }
    /* producer p forms chunk m NP + p of every round m */
    const int p = w - 1;
    double xi[TW], yi[TW], zi[TW];
    int iq[TW];
    bool okq[TW];
#pragma unroll
    for (int q = 0; q < TW; ++q) {
        okq[q] = q < it.ni;
        iq[q] = it.i0 + (okq[q] ? q : 0);
        const double2 p0 = d.pD[3 * iq[q]], p1 = d.pD[3 * iq[q] + 1];
        xi[q] = p0.x; yi[q] = p0.y; zi[q] = p1.x;
    }
    int bad = 0;
    constexpr int U = CW / 64; /* sources per lane and chunk */
    double2 s0[U], s1[U], s2[U]; /* the sources of the next chunk to form */
    auto load = [&](int k) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int lj = k * CW + u * 64 + l;
            const int j = off + (lj < Nb ? lj : Nb - 1);
            s0[u] = d.pD[3 * j];
            s1[u] = d.pD[3 * j + 1];
            s2[u] = d.pD[3 * j + 2];
        }
    };
    auto form = [&](int k, double* Tb0) {
        double rx[U][TW], ry[U][TW], rz[U][TW], r2s[U][TW], ir[U][TW];
        bool skip[U][TW];
        int safe = 1;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int lj = k * CW + u * 64 + l;
            const bool in = lj < Nb;
            const int j = off + lj;
#pragma unroll
            for (int q = 0; q < TW; ++q) {
                rx[u][q] = xi[q] - s0[u].x;
                ry[u][q] = yi[q] - s0[u].y;
                rz[u][q] = zi[q] - s1[u].x;
                const double r2 = (rx[u][q] * rx[u][q] + ry[u][q] * ry[u][q]) + rz[u][q] * rz[u][q];
                const bool self = j == iq[q];
                skip[u][q] = !in || self || r2 == 0.0;
                bad |= in && okq[q] && !self && r2 == 0.0;
                r2s[u][q] = skip[u][q] ? 1.0 : r2;
                safe &= f64_plain_range(r2s[u][q]);
            }
        }
        if (__all(safe)) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < TW; ++q) ir[u][q] = div_plain(1.0, sqrt_plain(r2s[u][q]));
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < TW; ++q) ir[u][q] = 1.0 / sqrt(r2s[u][q]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double* Tb = Tb0 + u * 64 + l;
            const double Fx = s1[u].y, Fy = s2[u].x, Fz = s2[u].y;
#pragma unroll
            for (int q = 0; q < TW; ++q) {
                const double fr = (rx[u][q] * Fx + ry[u][q] * Fy) + rz[u][q] * Fz;
                const double tt = fr / r2s[u][q];
                Tb[(0 * TW + q) * RS] = skip[u][q] ? 0.0 : ir[u][q] * (Fx + tt * rx[u][q]);
                Tb[(1 * TW + q) * RS] = skip[u][q] ? 0.0 : ir[u][q] * (Fy + tt * ry[u][q]);
                Tb[(2 * TW + q) * RS] = skip[u][q] ? 0.0 : ir[u][q] * (Fz + tt * rz[u][q]);
                if (RPY) {
                    const double ir3 = ir[u][q] / r2s[u][q];
                    const double t3 = 3.0 * tt;
                    Tb[(3 * TW + q) * RS] = skip[u][q] ? 0.0 : ir3 * (Fx - t3 * rx[u][q]);
                    Tb[(4 * TW + q) * RS] = skip[u][q] ? 0.0 : ir3 * (Fy - t3 * ry[u][q]);
                    Tb[(5 * TW + q) * RS] = skip[u][q] ? 0.0 : ir3 * (Fz - t3 * rz[u][q]);
                }
            }
        }
    };
    load(p);
    form(p, w_lds + p * BUF);
    load(NP + p);
    lds_barrier();
    for (int m = 0; m < M; ++m) {
        if (m + 1 < M) {
            form((m + 1) * NP + p, w_lds + (((m + 1) & 1) * NP + p) * BUF);
            load((m + 2) * NP + p);
        }
        lds_barrier();
    }
    if (__any(bad) && l == 0) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
}

/* Steric sum of sphere i over its candidate list (FP32C path). The list holds
 * every source that was closer than rc + skin at the previous stage; it is
 * sorted so that the terms are added in ascending j, exactly as the full
 * sum would add them, and then emptied for the next pair sum. */
__device__ int steric_list(const Dev& d, const Coef& c, int i, double acc[3], int* any) {
    const int N = d.Ntot;
    int n = d.nbr_cnt[i];
    n = n < NBR_CAP ? n : NBR_CAP; /* an overflow was flagged when it happened */
    n = n > 0 ? n : 0;
    int idx[NBR_CAP];
    for (int k = 0; k < n; ++k) {
        const int j = d.nbr_idx[i * NBR_CAP + k];
        idx[k] = (j >= 0 && j < N) ? j : i; /* entries come from the pair kernel; i itself is skipped */
    }
    for (int k = 1; k < n; ++k) { /* insertion sort, n <= NBR_CAP */
        const int v = idx[k];
        int m = k - 1;
        while (m >= 0 && idx[m] > v) {
            idx[m + 1] = idx[m];
            --m;
        }
        idx[m + 1] = v;
    }
    const double xi[3] = {d.Y[i], d.Y[N + i], d.Y[2 * N + i]};
    const double rc2 = c.rc * c.rc;
    int bad = 0;
    acc[0] = acc[1] = acc[2] = 0.0;
    *any = 0;
    for (int k = 0; k < n; ++k) {
        const int j = idx[k];
        if (j == i) continue;
        const double rx = xi[0] - d.Y[j], ry = xi[1] - d.Y[N + j], rz = xi[2] - d.Y[2 * N + j];
        const double r2 = (rx * rx + ry * ry) + rz * rz;
        if (r2 >= rc2) continue;
        if (r2 == 0.0) {
            bad = 1;
            continue;
        }
        const double r = sqrt(r2);
        const double cc = c.ks * (c.rc - r) / r;
        acc[0] = acc[0] + cc * rx;
        acc[1] = acc[1] + cc * ry;
        acc[2] = acc[2] + cc * rz;
        *any = 1;
    }
    d.nbr_cnt[i] = 0;
    return bad;
}

/* steric forces at the stage positions Y, then the pack: from the candidate
 * lists when the pair kernel records them, else by the full ascending sum */
__global__ void k_steric_pack(Dev d, Coef c, int prec) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.Stot) return;
    const int N = d.Ntot;
    const int i0 = 2 * s;
    double y0[3], y1[3], f0[3], f1[3];
    for (int a = 0; a < 3; ++a) {
        y0[a] = d.Y[a * N + i0];
        y1[a] = d.Y[a * N + i0 + 1];
        f0[a] = d.Fs[a * N + i0];
        f1[a] = d.Fs[a * N + i0 + 1];
    }
    double acc[3];
    int any, bad = 0;
    if (d.nbr_cnt) {
        bad |= steric_list(d, c, i0, acc, &any);
        if (any)
            for (int a = 0; a < 3; ++a) f0[a] = f0[a] + acc[a];
        bad |= steric_list(d, c, i0 + 1, acc, &any);
        if (any)
            for (int a = 0; a < 3; ++a) f1[a] = f1[a] + acc[a];
    } else {
        const int b = d.dsys[s];
        const int j0 = d.sys_off[b], j1 = d.sys_off[b + 1];
        auto get = [&](int j, double x[3]) {
            x[0] = d.Y[j];
            x[1] = d.Y[N + j];
            x[2] = d.Y[2 * N + j];
        };
        bad |= steric_sum(c, i0, j0, j1, get, acc, &any);
        if (any)
            for (int a = 0; a < 3; ++a) f0[a] = f0[a] + acc[a];
        bad |= steric_sum(c, i0 + 1, j0, j1, get, acc, &any);
        if (any)
            for (int a = 0; a < 3; ++a) f1[a] = f1[a] + acc[a];
    }
    if (bad) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
    store_pack(d, c, prec, i0, y0, y1, f0, f1, 1);
}

/* records: dumbbell centres and per-system mean position */
__global__ void k_record(Dev d, double* __restrict__ centres, double* __restrict__ com) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = d.Ntot;
    if (centres && g < d.Stot) {
        for (int a = 0; a < 3; ++a)
            centres[3 * g + a] = 0.5 * (d.X[a * N + 2 * g] + d.X[a * N + 2 * g + 1]);
    }
    if (com && g < 3 * d.nsys) {
        const int b = g / 3, a = g % 3;
        const int j0 = d.sys_off[b], j1 = d.sys_off[b + 1];
        double sum = 0.0;
        for (int j = j0; j < j1; ++j) sum = sum + d.X[a * N + j];
        com[3 * b + a] = sum / (double)(j1 - j0);
    }
}

/* ------------------------------------------------------- resident small systems */

/* Stage update of one component, in the operation order of stage_update,
 * with the RK accumulator r and the state x held by the caller. */
__device__ __forceinline__ double res_update(const Coef& c, int integ, int stage, int nst, double k, double& x,
                                             double& r, double nz) {
    double y;
    if (integ == 0) {
        if (stage == 0) {
            r = k;
            y = x + c.h2 * k;
        } else if (stage == 1) {
            r = r + 2.0 * k;
            y = x + c.h2 * k;
        } else if (stage == 2) {
            r = r + 2.0 * k;
            y = x + c.dt * k;
        } else {
            y = x + c.dt6 * (r + k);
        }
    } else {
        if (stage == 0) {
            r = k;
            y = x + c.dt * k;
        } else {
            y = x + c.h2 * (r + k);
        }
        if (c.noise) y = y + nz;
    }
    if (stage == nst - 1) x = y;
    return y;
}

/* Resident form (ad_launch.fused = 4): one work-group per system holds the
 * system on chip and runs every stage of nsteps steps in one launch, with
 * work-group barriers between the phases of a stage. The state comes from
 * and returns to d.X; the first stage's forces are formed at
 * (st0, ct0) = (sin, cos)(omega t) of step step0, and every later stage's
 * at the step table's row, the next step's row loaded while a step runs. */

/* One level of the fixed butterfly that combines the (hi, lo) sums
 * v = (hi.x, lo.x, hi.y, lo.y, hi.z, lo.z) of adjacent lanes: each lane takes
 * the sums of lane (itself xor distance) and adds them in with TwoSum. */
__device__ __forceinline__ void combine_hilo(float v[6], const float o[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float& hi = v[2 * a];
        float& lo = v[2 * a + 1];
        const float oh = o[2 * a], ol = o[2 * a + 1];
        const float s = hi + oh;
        const float bb = s - hi;
        const float err = (hi - (s - bb)) + (oh - bb);
        hi = s;
        lo = (lo + ol) + err;
    }
}
/* distances 1 and 2 through DPP quad permutations (CTRL 0xB1 swaps the lanes
 * of each pair, 0x4E the pairs of each quad): a VALU operation, no LDS round
 * trip */
template <int CTRL>
__device__ __forceinline__ void combine_level_dpp(float v[6]) {
    float o[6];
#pragma unroll
    for (int q = 0; q < 6; ++q)
        o[q] = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v[q]), CTRL, 0xF,
                                                                     0xF, false));
    combine_hilo(v, o);
}
/* larger distances (uniform over the wave) through ds_bpermute */
__device__ __forceinline__ void combine_level_shfl(float v[6], int sh) {
    float o[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) o[q] = __shfl_xor(v[q], sh);
    combine_hilo(v, o);
}

/* FP64 (the plain sum, bitwise that of the sequential oracle): X, R, Y, F
 * and the pair sums in LDS. Per stage: the terms of a chunk of source
 * columns are evaluated in parallel into an LDS matrix, then every
 * (target, component) thread adds its row of the chunk in ascending j;
 * the closing (velocity, stage update, next stage position) takes one
 * thread per sphere component, the next stage's spring forces one thread
 * per sphere (both threads of a dumbbell evaluate them from the same
 * inputs, so they agree bit for bit). */
template <int RPY, int INTEG>
__global__ __launch_bounds__(RES_T) void k_resident(Dev d, Epi e, long long step0, int nsteps, double st0,
                                                    double ct0) {
    /* INTEG: 0 RK4, 1 Heun, 2 Heun with noise; the stages are unrolled, so
     * every stage's update and table entries are fixed at compile time */
    constexpr int NST = INTEG == 0 ? 4 : 2;
    constexpr int T = RES_T;
    extern __shared__ double res_lds[];
    const Item it = d.fitems[blockIdx.x];
    const int n = it.Nb, ioff = it.ioff;
    const int N = d.Ntot;
    const int tid = threadIdx.x;
    const Coef& c = e.c;
    double* X = res_lds;
    double* R = X + 3 * n;
    double* Y = R + 3 * n;
    double* F = Y + 3 * n;
    double* Acc = F + 3 * n; /* pair sums [3][n] (RPY: then [3][n]) */
    double* Bcc = Acc + 3 * n;
    double* Tm = reinterpret_cast<double*>(reinterpret_cast<char*>(res_lds) +
                                           ((3 * n * (5 + (RPY ? 1 : 0))) * 8 + 15) / 16 * 16);
    const int cc = resident_cols(n, RPY);
    /* the chunk's terms [3][n][cs]: a row of cs (odd) doubles, so that the
     * threads of consecutive targets read distinct LDS banks */
    const int cs = resident_col_stride(cc);
    double* Tb = Tm + 3 * n * cs; /* RPY corrections of the chunk */

    for (int q = tid; q < 3 * n; q += T) {
        const int a = q / n, i = q - a * n;
        const double v = d.X[a * N + ioff + i];
        X[q] = v;
        Y[q] = v;
    }
    double2 tp = make_double2(0.0, 0.0);
    if (tid < n) tp = d.phitrig[(ioff >> 1) + (tid >> 1)];
    int bad = 0;
    /* the step table's row index in a vector register: its loads are then
     * vector loads, which the LDS-only barriers do not wait for */
    int row = (int)(step0 & (d.ring - 1));
    asm volatile("" : "+v"(row));
    double tb[8], nb[8];
    for (int q = 0; q < 8; ++q) tb[q] = nb[q] = 0.0;
    if (tid < n)
        for (int q = 0; q < 8; ++q) tb[q] = d.tab[row * 8 + q];
    __syncthreads();

    auto forces = [&](double st, double ct) {
        if (tid < n) {
            const int i0 = tid & ~1;
            double y0[3], y1[3], f0[3], f1[3];
            for (int a = 0; a < 3; ++a) {
                y0[a] = Y[a * n + i0];
                y1[a] = Y[a * n + i0 + 1];
            }
            spring_forces(c, y0, y1, tp.x, tp.y, st, ct, f0, f1);
            for (int a = 0; a < 3; ++a) F[a * n + tid] = (tid & 1) ? f1[a] : f0[a];
        }
        lds_barrier();
    };
    forces(st0, ct0);

    auto stage_pass = [&](auto stage_c, long long step) {
        constexpr int stage = decltype(stage_c)::value;
        for (int j0 = 0; j0 < n; j0 += cc) {
            const int nc = min(cc, n - j0);
            for (int p = tid; p < n * nc; p += T) {
                const int i = p / nc, jj = p - i * nc, j = j0 + jj;
                const int o = i * cs + jj;
                const int m = n * cs; /* component stride */
                const double r[3] = {Y[i] - Y[j], Y[n + i] - Y[n + j], Y[2 * n + i] - Y[2 * n + j]};
                const double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
                double t[3] = {0.0, 0.0, 0.0}, tq[3] = {0.0, 0.0, 0.0};
                if (j != i && r2 != 0.0) {
                    const double Fj[3] = {F[j], F[n + j], F[2 * n + j]};
                    oseen_term64(r, Fj, t);
                    if (RPY) rpy_term64(r, Fj, tq);
                } else if (j != i) {
                    bad = 1;
                }
                for (int a = 0; a < 3; ++a) {
                    Tm[a * m + o] = t[a];
                    if (RPY) Tb[a * m + o] = tq[a];
                }
            }
            lds_barrier();
            /* one thread per (component, target): the target's row of the
             * chunk in ascending j, its LDS loads eight at a time */
            for (int q = tid; q < 3 * n; q += T) {
                const double* row = Tm + q * cs; /* component q / n of target q mod n */
                const double* rowb = Tb + q * cs;
                /* The self term was stored as +0.0 and is added like the
                 * others: a sum that starts at +0.0 is never -0.0 in
                 * round-to-nearest, so adding +0.0 leaves it unchanged, bit
                 * for bit the sum that skips j = i. */
                double acc = (j0 == 0) ? 0.0 : Acc[q];
                double bcc = (RPY && j0 > 0) ? Bcc[q] : 0.0;
                int jb = 0;
                for (; jb + 8 <= nc; jb += 8) {
                    double v[8], w[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        v[u] = row[jb + u];
                        w[u] = RPY ? rowb[jb + u] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        acc = acc + v[u];
                        if (RPY) bcc = bcc + w[u];
                    }
                }
                for (; jb < nc; ++jb) {
                    acc = acc + row[jb];
                    if (RPY) bcc = bcc + rowb[jb];
                }
                Acc[q] = acc;
                if (RPY) Bcc[q] = bcc;
            }
            lds_barrier();
        }
        /* closing, one thread per (component, sphere) */
        for (int q = tid; q < 3 * n; q += T) {
            const int a = (q >= n) + (q >= 2 * n), i = q - a * n, o = q;
            double k = c.cs * F[o] + c.co * Acc[o];
            if (RPY) k = k + c.cr * Bcc[o];
            if (!isfinite(k)) bad = 1;
            const double nz = INTEG == 2 ? c.g * gauss_component(c.seed, ioff + i, step, a) : 0.0;
            double x = X[o], r = R[o];
            Y[o] = res_update(c, INTEG == 0 ? 0 : 1, stage, NST, k, x, r, nz);
            X[o] = x;
            R[o] = r;
        }
        lds_barrier();
        forces(tb[2 * stage], tb[2 * stage + 1]);
    };
    for (int sn = 0; sn < nsteps; ++sn) {
        const long long step = step0 + sn;
        row = row + 1 == d.ring ? 0 : row + 1;
        if (tid < n)
            for (int q = 0; q < 8; ++q) nb[q] = d.tab[row * 8 + q];
        stage_pass(std::integral_constant<int, 0>{}, step);
        stage_pass(std::integral_constant<int, 1>{}, step);
        if constexpr (NST == 4) {
            stage_pass(std::integral_constant<int, 2>{}, step);
            stage_pass(std::integral_constant<int, 3>{}, step);
        }
        for (int q = 0; q < 8; ++q) tb[q] = nb[q];
    }
    for (int q = tid; q < 3 * n; q += T) {
        const int a = q / n, i = q - a * n;
        d.X[a * N + ioff + i] = X[q];
    }
    if (__syncthreads_or(bad) && tid == 0) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
}

/* FP32C: the state in registers, only the float pack in LDS. Target sphere
 * t of the system has `split` adjacent lanes (a power of two <= 32, so a
 * dumbbell's lanes lie in one wave); lane 0 of them, the sphere's own lane,
 * holds its FP64 state x, RK accumulator r, stage position y and
 * self-and-partner velocity u0. Per stage:
 *   pair sums: each of the split lanes takes every split-th source in
 *   ascending order (own dumbbell masked by a zero 1/r), folding into
 *   (hi, lo) with TwoSum every 32 sources; the lanes are combined in a
 *   fixed butterfly;
 *   closing in the own lane: velocity, stage update, next stage position;
 *   next forces in the own lane: the partner's position by a lane exchange,
 *   the spring forces (both lanes of a dumbbell evaluate the same
 *   expression), u0 (the partner term reusing the spring's 1/d), and the
 *   sphere's pack entry, written into the other of two pack buffers;
 * then one work-group barrier. Stage s reads buffer s mod 2 and writes the
 * other, and every read of a buffer precedes the barrier that precedes its
 * next write. */
template <int SPLIT, int RPY, int T, int INTEG>
__global__ __launch_bounds__(T) void k_resident_c(Dev d, Epi e, long long step0, int nsteps, double st0,
                                                  double ct0) {
    /* INTEG: 0 RK4, 1 Heun, 2 Heun with noise; the stages are unrolled, so
     * every stage's update and table entries are fixed at compile time */
    constexpr int NST = INTEG == 0 ? 4 : 2;
    extern __shared__ float4 rc_lds[];
    const Item it = d.fitems[blockIdx.x];
    const int n = it.Nb, ioff = it.ioff;
    const int N = d.Ntot;
    const int tid = threadIdx.x;
    const Coef& c = e.c;
    const int split = resident_split(n, T);
    const int t = tid >> __builtin_ctz(split), sub = tid & (split - 1);
    const bool own = t < n && sub == 0;
    const int h = t & 1;
    const int pstride = resident_pack_f4(n); /* float4 per pack buffer */

    double x[3], r[3], y[3], u0[3];
    double2 tp = make_double2(0.0, 0.0);
    double tb[8], nb[8];
    for (int a = 0; a < 3; ++a) x[a] = r[a] = y[a] = u0[a] = 0.0;
    for (int q = 0; q < 8; ++q) tb[q] = nb[q] = 0.0;
    /* the step table's row index, held in a vector register so that its
     * loads are vector loads, which the LDS waits and barriers do not wait
     * for (a scalar load would be waited for by every LDS wait) */
    int row = (int)(step0 & (d.ring - 1));
    asm volatile("" : "+v"(row));
    if (own) {
        for (int a = 0; a < 3; ++a) x[a] = y[a] = d.X[a * N + ioff + t];
        tp = d.phitrig[(ioff >> 1) + (t >> 1)];
        for (int q = 0; q < 8; ++q) tb[q] = d.tab[row * 8 + q];
    }
    int bad = 0;

    auto forces = [&](double st, double ct, int buf) {
        double yp[3];
        for (int a = 0; a < 3; ++a) yp[a] = __shfl_xor(y[a], split);
        if (own) {
            /* lower and upper sphere of the dumbbell, by value selects (a
             * select of array pointers would put the arrays in scratch) */
            double ya[3], yb[3], f0[3], f1[3], f[3], fp[3];
            for (int a = 0; a < 3; ++a) {
                ya[a] = h ? yp[a] : y[a];
                yb[a] = h ? y[a] : yp[a];
            }
            const double id = spring_forces_rs(c, ya, yb, tp.x, tp.y, st, ct, f0, f1);
            for (int a = 0; a < 3; ++a) {
                f[a] = h ? f1[a] : f0[a];
                fp[a] = h ? f0[a] : f1[a];
            }
            /* r = y - yp is +-(y1 - y0) exactly, so 1/|r| is the spring's 1/d */
            const double rr[3] = {y[0] - yp[0], y[1] - yp[1], y[2] - yp[2]};
            const double ir2 = id * id;
            const double tt = ((rr[0] * fp[0] + rr[1] * fp[1]) + rr[2] * fp[2]) * ir2;
            for (int a = 0; a < 3; ++a) {
                double u = c.cs * f[a] + c.co * (id * (fp[a] + tt * rr[a]));
                if (RPY) u = u + c.cr * ((id * ir2) * (fp[a] - (3.0 * tt) * rr[a]));
                u0[a] = u;
            }
            float hi[3], lo[3];
            for (int a = 0; a < 3; ++a) split_f32(y[a], hi[a], lo[a]);
            float4* pA = rc_lds + buf * pstride;
            float4* pB = pA + n;
            float* pz = reinterpret_cast<float*>(pB + n);
            pA[t] = make_float4(hi[0], hi[1], hi[2], (float)f[0]);
            pB[t] = make_float4(lo[0], lo[1], lo[2], (float)f[1]);
            pz[t] = (float)f[2];
        }
        lds_barrier();
    };

    int buf = 0;
    forces(st0, ct0, buf);
    const float crr = c.crr;
    auto stage_pass = [&](auto stage_c, long long step) {
        constexpr int stage = decltype(stage_c)::value;
        const float4* pA = rc_lds + buf * pstride;
        const float4* pB = pA + n;
        const float* pz = reinterpret_cast<const float*>(pB + n);
        float ax = 0.f, ay = 0.f, az = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
        if (t < n) {
            const float4 Ai = pA[t];
            const float4 Bi = pB[t];
            const int dt = t >> 1;
            float px = 0.f, py = 0.f, pzz = 0.f;
            int cnt = 0;
            /* four sources at a time, their LDS loads issued together; the
             * own dumbbell and the sources past the end are masked by a zero
             * 1/r (their term is then exactly zero) */
            for (int j0 = sub; j0 < n; j0 += 4 * split) {
                float4 Aj[4], Bj[4];
                float Fz[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = j0 + u * split;
                    const int jj = j < n ? j : t;
                    Aj[u] = pA[jj];
                    Bj[u] = pB[jj];
                    Fz[u] = pz[jj];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = j0 + u * split;
                    float rx, ry, rz;
                    if (SPLIT) {
                        rx = (Ai.x - Aj[u].x) + (Bi.x - Bj[u].x);
                        ry = (Ai.y - Aj[u].y) + (Bi.y - Bj[u].y);
                        rz = (Ai.z - Aj[u].z) + (Bi.z - Bj[u].z);
                    } else {
                        rx = Ai.x - Aj[u].x;
                        ry = Ai.y - Aj[u].y;
                        rz = Ai.z - Aj[u].z;
                    }
                    const float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
                    float ir = __builtin_amdgcn_rsqf(r2);
                    if (j >= n || (j >> 1) == dt) ir = 0.f;
                    pair_term<RPY>(ir, rx, ry, rz, Aj[u].w, Bj[u].w, Fz[u], crr, px, py, pzz);
                }
                cnt += 4;
                if (cnt == 32) {
                    two_sum_acc(ax, bx, px);
                    two_sum_acc(ay, by, py);
                    two_sum_acc(az, bz, pzz);
                    px = py = pzz = 0.f;
                    cnt = 0;
                }
            }
            two_sum_acc(ax, bx, px);
            two_sum_acc(ay, by, py);
            two_sum_acc(az, bz, pzz);
        }
        float v[6] = {ax, bx, ay, by, az, bz};
        if (split > 1) combine_level_dpp<0xB1>(v);
        if (split > 2) combine_level_dpp<0x4E>(v);
        for (int sh = 4; sh < split; sh *= 2) combine_level_shfl(v, sh);
        if (own) {
            const double acc[3] = {(double)v[0] + (double)v[1], (double)v[2] + (double)v[3],
                                   (double)v[4] + (double)v[5]};
            for (int a = 0; a < 3; ++a) {
                const double k = u0[a] + c.co * acc[a];
                if (!isfinite(k)) bad = 1;
                const double nz = INTEG == 2 ? c.g * gauss_component(c.seed, ioff + t, step, a) : 0.0;
                y[a] = res_update(c, INTEG == 0 ? 0 : 1, stage, NST, k, x[a], r[a], nz);
            }
        }
        buf ^= 1;
        forces(tb[2 * stage], tb[2 * stage + 1], buf);
    };
    for (int sn = 0; sn < nsteps; ++sn) {
        const long long step = step0 + sn;
        row = row + 1 == d.ring ? 0 : row + 1;
        if (own)
            for (int q = 0; q < 8; ++q) nb[q] = d.tab[row * 8 + q];
        stage_pass(std::integral_constant<int, 0>{}, step);
        stage_pass(std::integral_constant<int, 1>{}, step);
        if constexpr (NST == 4) {
            stage_pass(std::integral_constant<int, 2>{}, step);
            stage_pass(std::integral_constant<int, 3>{}, step);
        }
        for (int q = 0; q < 8; ++q) tb[q] = nb[q];
    }
    if (own)
        for (int a = 0; a < 3; ++a) d.X[a * N + ioff + t] = x[a];
    if (__syncthreads_or(bad) && tid == 0) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
}

/* ------------------------------------------------------------ launchers */

static inline dim3 blocks_for(int n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

hipError_t launch_set_step(const Dev& d, long long step, hipStream_t s) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, d.ctl, step);
    return hipGetLastError();
}

hipError_t launch_clear_flag(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, s, d.ctl);
    return hipGetLastError();
}

hipError_t launch_clear_counts(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_counts, blocks_for(d.Ntot, 256), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_state_in(const Dev& d, const double* Xa, hipStream_t s) {
    hipLaunchKernelGGL(k_state_in, blocks_for(d.Ntot, 256), dim3(256), 0, s, d, Xa);
    return hipGetLastError();
}

hipError_t launch_state_out(const Dev& d, double* Xa, hipStream_t s) {
    hipLaunchKernelGGL(k_state_out, blocks_for(d.Ntot, 256), dim3(256), 0, s, d, Xa);
    return hipGetLastError();
}

hipError_t launch_pack_state(const Dev& d, const Coef& c, int prec, double st, double ct, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_state, blocks_for(d.Stot, 128), dim3(128), 0, s, d, c, prec, st, ct);
    return hipGetLastError();
}

hipError_t launch_pack_apply(const Dev& d, const Coef& c, int prec, const double* Xa, const double* Fa,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_pack_apply, blocks_for(d.Stot, 128), dim3(128), 0, s, d, c, prec, Xa, Fa);
    return hipGetLastError();
}

hipError_t launch_forces(const Dev& d, const Coef& c, const double* Xa, double st, double ct, double* Fa,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_forces, blocks_for(d.Stot, 128), dim3(128), 0, s, d, c, Xa, st, ct, Fa);
    return hipGetLastError();
}

/* Launch a pair kernel; with timing events the launch goes through
 * hipExtLaunchKernelGGL, whose events carry the dispatch's own start and end
 * times. */
struct Timing {
    hipEvent_t start, stop;
};

template <class K>
static hipError_t go(K kern, int wg, const Dev& d, const Epi& e, int mode, hipStream_t s, const Timing& tm) {
    if (tm.start)
        hipExtLaunchKernelGGL(kern, dim3(d.nitems), dim3(wg), 0, s, tm.start, tm.stop, 0, d, e, mode);
    else
        hipLaunchKernelGGL(kern, dim3(d.nitems), dim3(wg), 0, s, d, e, mode);
    return hipGetLastError();
}

template <int WG, int WJ, int SPLIT, int STERIC, int RPY>
static hipError_t f32c_ipl(const Dev& d, const Epi& e, int ipl, int mode, hipStream_t s, const Timing& tm) {
    if (ipl == 1) return go(k_pairs_f32c<WG, 1, WJ, SPLIT, STERIC, RPY>, WG, d, e, mode, s, tm);
    if (ipl == 2) return go(k_pairs_f32c<WG, 2, WJ, SPLIT, STERIC, RPY>, WG, d, e, mode, s, tm);
    if (ipl == 4) return go(k_pairs_f32c<WG, 4, WJ, SPLIT, STERIC, RPY>, WG, d, e, mode, s, tm);
    return hipErrorInvalidValue;
}

template <int WG, int WJ, int RPY>
static hipError_t f32c_var(const Dev& d, const Epi& e, const Shape& sh, int mode, hipStream_t s, const Timing& tm) {
    if (sh.steric)
        return sh.split ? f32c_ipl<WG, WJ, 1, 1, RPY>(d, e, sh.ipl, mode, s, tm)
                        : f32c_ipl<WG, WJ, 0, 1, RPY>(d, e, sh.ipl, mode, s, tm);
    return sh.split ? f32c_ipl<WG, WJ, 1, 0, RPY>(d, e, sh.ipl, mode, s, tm)
                    : f32c_ipl<WG, WJ, 0, 0, RPY>(d, e, sh.ipl, mode, s, tm);
}

template <int WG, int WJ>
static hipError_t f32c_ten(const Dev& d, const Epi& e, const Shape& sh, int mode, hipStream_t s, const Timing& tm) {
    return sh.rpy ? f32c_var<WG, WJ, 1>(d, e, sh, mode, s, tm) : f32c_var<WG, WJ, 0>(d, e, sh, mode, s, tm);
}

template <int WG, int IPL>
static hipError_t f64_ten(const Dev& d, const Epi& e, const Shape& sh, int mode, hipStream_t s, const Timing& tm) {
    return sh.rpy ? go(k_pairs_f64<WG, IPL, 1>, WG, d, e, mode, s, tm) : go(k_pairs_f64<WG, IPL, 0>, WG, d, e, mode, s, tm);
}

template <int TW, int CW>
static hipError_t go_f64w(const Dev& d, const Epi& e, const Shape& sh, int mode, hipStream_t s, const Timing& tm) {
    constexpr int NP = F64W_NP;
    auto kern = sh.rpy ? k_pairs_f64w<TW, NP, CW, 1> : k_pairs_f64w<TW, NP, CW, 0>;
    const size_t lds = f64w_lds_bytes(TW, sh.rpy, CW);
    const dim3 block(64 * (NP + 1));
    if (tm.start)
        hipExtLaunchKernelGGL(kern, dim3(d.nfitems), block, lds, s, tm.start, tm.stop, 0, d, e, mode);
    else
        hipLaunchKernelGGL(kern, dim3(d.nfitems), block, lds, s, d, e, mode);
    return hipGetLastError();
}

hipError_t launch_pairs(const Dev& d, const Epi& e, const Shape& sh, int mode, hipStream_t s, hipEvent_t ev_start,
                        hipEvent_t ev_stop) {
    if (d.nitems <= 0) return hipSuccess;
    const Timing tm{ev_start, ev_stop};
    if (e.prec == PREC_FP32C) {
        if (sh.steric && !d.nbr_cnt) return hipErrorInvalidValue;
        if (sh.wg == 64 && sh.wj == 1) return f32c_ten<64, 1>(d, e, sh, mode, s, tm);
        if (sh.wg == 256 && sh.wj == 1) return f32c_ten<256, 1>(d, e, sh, mode, s, tm);
        if (sh.wg == 256 && sh.wj == 4) return f32c_ten<256, 4>(d, e, sh, mode, s, tm);
        return hipErrorInvalidValue;
    }
    /* AD_FP64: the terms spread over waves (work list of target blocks) */
    if (e.prec == PREC_FP64 && d.nfitems > 0) {
        const int tw = f64w_targets(d.Ntot);
        if (tw == 4)
            return f64w_chunk(d.Ntot) == 128 ? go_f64w<4, 128>(d, e, sh, mode, s, tm)
                                             : go_f64w<4, 64>(d, e, sh, mode, s, tm);
        if (tw == 2) return go_f64w<2, 64>(d, e, sh, mode, s, tm);
        return go_f64w<1, 64>(d, e, sh, mode, s, tm);
    }
    /* FP64 kernels: 1 or 2 targets per lane, no j split inside a group; the
     * work list was built for this shape, so anything else is refused */
    if (sh.wj != 1) return hipErrorInvalidValue;
    if (sh.wg == 64 && sh.ipl == 1) return f64_ten<64, 1>(d, e, sh, mode, s, tm);
    if (sh.wg == 64 && sh.ipl == 2) return f64_ten<64, 2>(d, e, sh, mode, s, tm);
    if (sh.wg == 256 && sh.ipl == 1) return f64_ten<256, 1>(d, e, sh, mode, s, tm);
    if (sh.wg == 256 && sh.ipl == 2) return f64_ten<256, 2>(d, e, sh, mode, s, tm);
    return hipErrorInvalidValue;
}

template <int SPLIT, int RPY, int NW>
static hipError_t go_fused(const Dev& d, const Epi& e, int maxNb, hipStream_t s, const Timing& tm) {
    const int lds = fused_lds_bytes(maxNb, SPLIT, NW);
    const dim3 grid(d.nfitems ? d.nfitems : (d.Ntot + FS_I - 1) / FS_I);
    auto kern = k_stage_fused<SPLIT, RPY, NW>;
    if (tm.start)
        hipExtLaunchKernelGGL(kern, grid, dim3(64 * NW), lds, s, tm.start, tm.stop, 0, d, e);
    else
        hipLaunchKernelGGL(kern, grid, dim3(64 * NW), lds, s, d, e);
    return hipGetLastError();
}

template <int SPLIT, int RPY>
static hipError_t go_wide(const Dev& d, const Epi& e, int maxNb, hipStream_t s, const Timing& tm) {
    const int lds = fused_wide_lds_bytes(maxNb, SPLIT);
    auto kern = k_stage_wide<SPLIT, RPY>;
    if (tm.start)
        hipExtLaunchKernelGGL(kern, dim3(d.nfitems), dim3(256), lds, s, tm.start, tm.stop, 0, d, e);
    else
        hipLaunchKernelGGL(kern, dim3(d.nfitems), dim3(256), lds, s, d, e);
    return hipGetLastError();
}

template <int SPLIT, int RPY>
static hipError_t go_stream(const Dev& d, const Epi& e, hipStream_t s, const Timing& tm) {
    const int ti = stream_targets(d.Ntot), nw = stream_waves(ti);
    const int lds = fused_stream_lds_bytes(SPLIT, nw, ti);
    const dim3 grid(d.nfitems ? d.nfitems : (d.Ntot + ti - 1) / ti);
    auto kern = ti == 16 ? (grid.x > 256 ? k_stage_stream_x2<SPLIT, RPY, 16, 16> : k_stage_stream<SPLIT, RPY, 16, 16>)
                : ti == 8 ? k_stage_stream<SPLIT, RPY, 8, 8> : k_stage_stream<SPLIT, RPY, 4, 8>;
    if (tm.start)
        hipExtLaunchKernelGGL(kern, grid, dim3(64 * nw), lds, s, tm.start, tm.stop, 0, d, e);
    else
        hipLaunchKernelGGL(kern, grid, dim3(64 * nw), lds, s, d, e);
    return hipGetLastError();
}

template <int RPY>
static hipError_t go_stream64(const Dev& d, const Epi& e, hipStream_t s, const Timing& tm) {
    const int lds = fused_stream64_lds_bytes();
    const int ti = stream_targets(d.Ntot);
    const dim3 grid(d.nfitems ? d.nfitems : (d.Ntot + ti - 1) / ti);
    auto kern = ti == 16 ? k_stage_stream64<RPY, 16> : ti == 8 ? k_stage_stream64<RPY, 8> : k_stage_stream64<RPY, 4>;
    if (tm.start)
        hipExtLaunchKernelGGL(kern, grid, dim3(1024), lds, s, tm.start, tm.stop, 0, d, e);
    else
        hipLaunchKernelGGL(kern, grid, dim3(1024), lds, s, d, e);
    return hipGetLastError();
}

typedef void (*ResidentKernel)(Dev, Epi, long long, int, double, double);

template <int SPLIT, int RPY, int T>
static ResidentKernel resident_c_integ(int integ) {
    if (integ == 0) return k_resident_c<SPLIT, RPY, T, 0>;
    if (integ == 1) return k_resident_c<SPLIT, RPY, T, 1>;
    return k_resident_c<SPLIT, RPY, T, 2>;
}

template <int T>
static ResidentKernel resident_c_threads(int hilo, int rpy, int integ) {
    if (hilo) return rpy ? resident_c_integ<1, 1, T>(integ) : resident_c_integ<1, 0, T>(integ);
    return rpy ? resident_c_integ<0, 1, T>(integ) : resident_c_integ<0, 0, T>(integ);
}

/* the FP32C resident kernel for hi/lo positions or not, RPY or not, T
 * threads (64, 128, 256 or 512) and integrator integ (0 RK4, 1 Heun, 2 Heun
 * with noise) */
static ResidentKernel resident_c_kernel(int hilo, int rpy, int T, int integ) {
    switch (T) {
        case 64: return resident_c_threads<64>(hilo, rpy, integ);
        case 128: return resident_c_threads<128>(hilo, rpy, integ);
        case 256: return resident_c_threads<256>(hilo, rpy, integ);
        default: return resident_c_threads<512>(hilo, rpy, integ);
    }
}

hipError_t prepare_fused() {
    const void* kernels[] = {reinterpret_cast<const void*>(&k_stage_stream<0, 0, 16, 16>),
                             reinterpret_cast<const void*>(&k_stage_stream<0, 1, 16, 16>),
                             reinterpret_cast<const void*>(&k_stage_stream<1, 0, 16, 16>),
                             reinterpret_cast<const void*>(&k_stage_stream<1, 1, 16, 16>),
                             reinterpret_cast<const void*>(&k_stage_stream_x2<0, 0, 16, 16>),
                             reinterpret_cast<const void*>(&k_stage_stream_x2<0, 1, 16, 16>),
                             reinterpret_cast<const void*>(&k_stage_stream_x2<1, 0, 16, 16>),
                             reinterpret_cast<const void*>(&k_stage_stream_x2<1, 1, 16, 16>),
                             reinterpret_cast<const void*>(&k_stage_stream<0, 0, 8, 8>),
                             reinterpret_cast<const void*>(&k_stage_stream<0, 1, 8, 8>),
                             reinterpret_cast<const void*>(&k_stage_stream<1, 0, 8, 8>),
                             reinterpret_cast<const void*>(&k_stage_stream<1, 1, 8, 8>),
                             reinterpret_cast<const void*>(&k_stage_stream<0, 0, 4, 8>),
                             reinterpret_cast<const void*>(&k_stage_stream<0, 1, 4, 8>),
                             reinterpret_cast<const void*>(&k_stage_stream<1, 0, 4, 8>),
                             reinterpret_cast<const void*>(&k_stage_stream<1, 1, 4, 8>),
                             reinterpret_cast<const void*>(&k_stage_stream64<0, 16>),
                             reinterpret_cast<const void*>(&k_stage_stream64<1, 16>),
                             reinterpret_cast<const void*>(&k_stage_stream64<0, 8>),
                             reinterpret_cast<const void*>(&k_stage_stream64<1, 8>),
                             reinterpret_cast<const void*>(&k_stage_stream64<0, 4>),
                             reinterpret_cast<const void*>(&k_stage_stream64<1, 4>),
                             reinterpret_cast<const void*>(&k_stage_wide<0, 0>),
                             reinterpret_cast<const void*>(&k_stage_wide<0, 1>),
                             reinterpret_cast<const void*>(&k_stage_wide<1, 0>),
                             reinterpret_cast<const void*>(&k_stage_wide<1, 1>),
                             reinterpret_cast<const void*>(&k_stage_fused<0, 0, 16>),
                             reinterpret_cast<const void*>(&k_stage_fused<0, 1, 16>),
                             reinterpret_cast<const void*>(&k_stage_fused<1, 0, 16>),
                             reinterpret_cast<const void*>(&k_stage_fused<1, 1, 16>),
                             reinterpret_cast<const void*>(&k_stage_fused<0, 0, 4>),
                             reinterpret_cast<const void*>(&k_stage_fused<0, 1, 4>),
                             reinterpret_cast<const void*>(&k_stage_fused<1, 0, 4>),
                             reinterpret_cast<const void*>(&k_stage_fused<1, 1, 4>)};
    for (const void* k : kernels) {
        hipError_t err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, FUSED_LDS_MAX);
        if (err != hipSuccess) {
            (void)hipGetLastError(); /* a later launch check must not report it again */
            return err;
        }
    }
    const void* resident[54] = {
        reinterpret_cast<const void*>(&k_resident<0, 0>), reinterpret_cast<const void*>(&k_resident<1, 0>),
        reinterpret_cast<const void*>(&k_resident<0, 1>), reinterpret_cast<const void*>(&k_resident<1, 1>),
        reinterpret_cast<const void*>(&k_resident<0, 2>), reinterpret_cast<const void*>(&k_resident<1, 2>)};
    for (int q = 0; q < 48; ++q)
        resident[6 + q] = reinterpret_cast<const void*>(
            resident_c_kernel(q & 1, (q >> 1) & 1, 64 << ((q >> 2) & 3), q >> 4));
    for (const void* k : resident) {
        hipError_t err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, RES_LDS_MAX);
        if (err != hipSuccess) {
            (void)hipGetLastError();
            return err;
        }
    }
    return hipSuccess;
}

hipError_t launch_resident(const Dev& d, const Epi& e, int hilo, int maxNb, long long step0, int nsteps,
                           double st0, double ct0, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop) {
    if (d.nfitems <= 0 || nsteps <= 0) return hipErrorInvalidValue;
    const int p64 = e.prec != PREC_FP32C;
    const int rpy = e.c.rpy;
    if (maxNb > (p64 ? RES_MAX64 : RES_MAX32)) return hipErrorInvalidValue;
    const size_t lds = (size_t)resident_lds_bytes(maxNb, p64, rpy);
    if (lds > (size_t)RES_LDS_MAX) return hipErrorInvalidValue;
    const int T = resident_threads(maxNb, p64);
    ResidentKernel kern;
    const int integ = e.integ == 0 ? 0 : (e.c.noise ? 2 : 1);
    if (p64)
        kern = integ == 0 ? (rpy ? k_resident<1, 0> : k_resident<0, 0>)
               : integ == 1 ? (rpy ? k_resident<1, 1> : k_resident<0, 1>)
                            : (rpy ? k_resident<1, 2> : k_resident<0, 2>);
    else
        kern = resident_c_kernel(hilo, rpy, T, integ);
    if (ev_start)
        hipExtLaunchKernelGGL(kern, dim3(d.nfitems), dim3(T), lds, s, ev_start, ev_stop, 0, d, e, step0, nsteps, st0,
                              ct0);
    else
        hipLaunchKernelGGL(kern, dim3(d.nfitems), dim3(T), lds, s, d, e, step0, nsteps, st0, ct0);
    return hipGetLastError();
}

hipError_t launch_fused(const Dev& d, const Epi& e, const Shape& sh, int maxNb, hipStream_t s,
                        hipEvent_t ev_start, hipEvent_t ev_stop) {
    const Timing tm0{ev_start, ev_stop};
    if (e.prec == PREC_FP64_TILED && sh.fused == 3 && !sh.steric && maxNb >= 2) {
        if ((d.nsys > 1) != (d.nfitems > 0)) return hipErrorInvalidValue;
        return sh.rpy ? go_stream64<1>(d, e, s, tm0) : go_stream64<0>(d, e, s, tm0);
    }
    if (e.prec != PREC_FP32C || sh.steric || maxNb < 2) return hipErrorInvalidValue;
    if (sh.fused == 2) {
        /* every work-group takes its (system, 64-target block) from the list */
        if (d.nfitems <= 0 || fused_wide_lds_bytes(maxNb, sh.split) > FUSED_LDS_MAX) return hipErrorInvalidValue;
        if (sh.split) return sh.rpy ? go_wide<1, 1>(d, e, maxNb, s, tm0) : go_wide<1, 0>(d, e, maxNb, s, tm0);
        return sh.rpy ? go_wide<0, 1>(d, e, maxNb, s, tm0) : go_wide<0, 0>(d, e, maxNb, s, tm0);
    }
    if ((d.nsys > 1) != (d.nfitems > 0)) return hipErrorInvalidValue;
    if (sh.fused == 3) {
        if (sh.split) return sh.rpy ? go_stream<1, 1>(d, e, s, tm0) : go_stream<1, 0>(d, e, s, tm0);
        return sh.rpy ? go_stream<0, 1>(d, e, s, tm0) : go_stream<0, 0>(d, e, s, tm0);
    }
    if (sh.fused != 1) return hipErrorInvalidValue;
    const int nw = d.nsys > 1 ? 4 : 16;
    if (fused_lds_bytes(maxNb, sh.split, nw) > FUSED_LDS_MAX) return hipErrorInvalidValue;
    const Timing tm{ev_start, ev_stop};
    if (nw == 16) {
        if (sh.split) return sh.rpy ? go_fused<1, 1, 16>(d, e, maxNb, s, tm) : go_fused<1, 0, 16>(d, e, maxNb, s, tm);
        return sh.rpy ? go_fused<0, 1, 16>(d, e, maxNb, s, tm) : go_fused<0, 0, 16>(d, e, maxNb, s, tm);
    }
    if (sh.split) return sh.rpy ? go_fused<1, 1, 4>(d, e, maxNb, s, tm) : go_fused<1, 0, 4>(d, e, maxNb, s, tm);
    return sh.rpy ? go_fused<0, 1, 4>(d, e, maxNb, s, tm) : go_fused<0, 0, 4>(d, e, maxNb, s, tm);
}

hipError_t launch_epilogue(const Dev& d, const Epi& e, hipStream_t s) {
    hipLaunchKernelGGL(k_epilogue, blocks_for(d.Ntot, EPI_S), dim3(EPI_T), 0, s, d, e);
    return hipGetLastError();
}

hipError_t launch_steric_pack(const Dev& d, const Coef& c, int prec, hipStream_t s) {
    hipLaunchKernelGGL(k_steric_pack, blocks_for(d.Stot, 128), dim3(128), 0, s, d, c, prec);
    return hipGetLastError();
}

hipError_t launch_record(const Dev& d, double* centres, double* com, hipStream_t s) {
    int n = d.Stot > 3 * d.nsys ? d.Stot : 3 * d.nsys;
    hipLaunchKernelGGL(k_record, blocks_for(n, 128), dim3(128), 0, s, d, centres, com);
    return hipGetLastError();
}

}  // namespace ad
