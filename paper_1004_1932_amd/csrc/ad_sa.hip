/*
 * Stroke-averaged far-field equations of motion on gfx950 (Putz, Dunkel,
 * Yeomans, Sec. III, Eqs. e:eom, J, K and the projections s, r, q):
 *   dR_s/dt = sum_{r != s} J^{sr},   dN_s/dt = -(I - N_s N_s) sum_{r != s} K^{sr},
 *   J^{sr} = a w sin(phi_s - phi_r) (9/64) (lam/ell)^2 (ell/D)^4
 *            { N_s (2s + 4qr - 10 s r^2)
 *              + Dhat (1 + 2q^2 - 5s^2 - 5r^2 - 20 q s r + 35 s^2 r^2) },
 *   K^{sr} = w sin(phi_s - phi_r) (15/64) (a/ell) (lam/ell)^2 (ell/D)^5 Dhat
 *            (3s + 6rq + 6 s q^2 - 7 s^3 - 21 s r^2 - 42 q s^2 r + 63 s^3 r^2),
 *   D = R_s - R_r, s = Dhat.N_s, r = Dhat.N_r, q = N_s.N_r.
 * One wave per dumbbell: lane l sums over the others j = l, l + 64, ... in
 * ascending order, and a fixed butterfly of shuffles adds the 64 partial
 * sums (every lane ends with the same bits). FP64 throughout, no FMA
 * contraction. (One thread per dumbbell left the paper's arrays of 125-729
 * dumbbells with one to six work-groups on the whole chip.)
 * A step is four launches of k_sa_stage (RK4); each also applies its stage's
 * update to its own dumbbell, and the last one scales the axes back to unit
 * length.
 */
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/ad.h"

namespace ad_sa {

constexpr double kPi = 3.14159265358979323846;
constexpr int SA_WG = 64; /* one wave, one dumbbell */

struct SaCoef {
    double ell, cj, ck; /* cj = a w (9/64)(lam/ell)^2, ck = w (15/64)(a/ell)(lam/ell)^2 */
    double h2, dt, dt6;
};

/* rates of dumbbell i against all S, reading positions Rs and axes Ns; called
 * by all 64 lanes of the wave that owns i, which all return the rates */
__device__ void sa_rates(const SaCoef& k, int S, int i, const double* __restrict__ Rs,
                         const double* __restrict__ Ns, const double* __restrict__ phi, double dR[3], double dN[3],
                         int* bad) {
    const int l = threadIdx.x & 63;
    double ri[3], ni[3];
    for (int a = 0; a < 3; ++a) {
        ri[a] = Rs[3 * i + a];
        ni[a] = Ns[3 * i + a];
    }
    const double pi_ = phi[i];
    double jx = 0.0, jy = 0.0, jz = 0.0, kx = 0.0, ky = 0.0, kz = 0.0;
    for (int j = l; j < S; j += 64) {
        if (j == i) continue;
        const double rj[3] = {Rs[3 * j], Rs[3 * j + 1], Rs[3 * j + 2]};
        const double nj[3] = {Ns[3 * j], Ns[3 * j + 1], Ns[3 * j + 2]};
        const double Dx = ri[0] - rj[0];
        const double Dy = ri[1] - rj[1];
        const double Dz = ri[2] - rj[2];
        const double D = sqrt((Dx * Dx + Dy * Dy) + Dz * Dz);
        if (D == 0.0) {
            *bad = 1;
            continue;
        }
        const double ux = Dx / D, uy = Dy / D, uz = Dz / D;
        const double s = (ux * ni[0] + uy * ni[1]) + uz * ni[2];
        const double r = (ux * nj[0] + uy * nj[1]) + uz * nj[2];
        const double q = (ni[0] * nj[0] + ni[1] * nj[1]) + ni[2] * nj[2];
        const double sn = sin(pi_ - phi[j]);
        const double x = k.ell / D;
        const double x4 = (x * x) * (x * x);
        const double aN = 2.0 * s + 4.0 * q * r - 10.0 * s * r * r;
        const double aD =
            1.0 + 2.0 * q * q - 5.0 * s * s - 5.0 * r * r - 20.0 * q * s * r + 35.0 * s * s * r * r;
        const double fj = k.cj * sn * x4;
        jx = jx + fj * (ni[0] * aN + ux * aD);
        jy = jy + fj * (ni[1] * aN + uy * aD);
        jz = jz + fj * (ni[2] * aN + uz * aD);
        const double bK = 3.0 * s + 6.0 * r * q + 6.0 * s * q * q - 7.0 * s * s * s - 21.0 * s * r * r -
                          42.0 * q * s * s * r + 63.0 * s * s * s * r * r;
        const double fk = k.ck * sn * (x4 * x) * bK;
        kx = kx + fk * ux;
        ky = ky + fk * uy;
        kz = kz + fk * uz;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        jx = jx + __shfl_xor(jx, o);
        jy = jy + __shfl_xor(jy, o);
        jz = jz + __shfl_xor(jz, o);
        kx = kx + __shfl_xor(kx, o);
        ky = ky + __shfl_xor(ky, o);
        kz = kz + __shfl_xor(kz, o);
    }
    dR[0] = jx;
    dR[1] = jy;
    dR[2] = jz;
    const double nk = (ni[0] * kx + ni[1] * ky) + ni[2] * kz;
    dN[0] = -(kx - ni[0] * nk);
    dN[1] = -(ky - ni[1] * nk);
    dN[2] = -(kz - ni[2] * nk);
}

__global__ __launch_bounds__(SA_WG) void k_sa_rhs(SaCoef k, int S, const double* __restrict__ R,
                                                  const double* __restrict__ N, const double* __restrict__ phi,
                                                  double* __restrict__ dR, double* __restrict__ dN, int* flag) {
    const int i = blockIdx.x; /* the grid has exactly S work-groups */
    double r[3], n[3];
    int bad = 0;
    sa_rates(k, S, i, R, N, phi, r, n, &bad);
    const int any = __any(bad);
    if (threadIdx.x != 0) return;
    for (int a = 0; a < 3; ++a) {
        dR[3 * i + a] = r[a];
        dN[3 * i + a] = n[a];
    }
    if (any && flag) atomicOr(flag, 1);
}

/* One RK4 stage: rates at the stage positions (YR, YN), accumulate, and write
 * the next stage positions (or, at the last stage, the new state). */
__global__ __launch_bounds__(SA_WG) void k_sa_stage(SaCoef k, int S, int stage, double* __restrict__ R,
                                                    double* __restrict__ N, const double* __restrict__ phi,
                                                    const double* __restrict__ YR, const double* __restrict__ YN,
                                                    double* __restrict__ ZR, double* __restrict__ ZN,
                                                    double* __restrict__ AR, double* __restrict__ AN, int* flag) {
    const int i = blockIdx.x; /* the grid has exactly S work-groups */
    double kr[3], kn[3];
    int bad = 0;
    sa_rates(k, S, i, YR, YN, phi, kr, kn, &bad);
    const int any = __any(bad);
    if (threadIdx.x != 0) return;
    if (any) atomicOr(flag, 1);
    double nv[3];
    for (int a = 0; a < 3; ++a) {
        const int o = 3 * i + a;
        const double x = R[o], v = N[o];
        if (stage == 0) {
            AR[o] = kr[a];
            AN[o] = kn[a];
            ZR[o] = x + k.h2 * kr[a];
            ZN[o] = v + k.h2 * kn[a];
        } else if (stage == 1) {
            AR[o] = AR[o] + 2.0 * kr[a];
            AN[o] = AN[o] + 2.0 * kn[a];
            ZR[o] = x + k.h2 * kr[a];
            ZN[o] = v + k.h2 * kn[a];
        } else if (stage == 2) {
            AR[o] = AR[o] + 2.0 * kr[a];
            AN[o] = AN[o] + 2.0 * kn[a];
            ZR[o] = x + k.dt * kr[a];
            ZN[o] = v + k.dt * kn[a];
        } else {
            R[o] = x + k.dt6 * (AR[o] + kr[a]);
            nv[a] = v + k.dt6 * (AN[o] + kn[a]);
        }
    }
    if (stage == 3) {
        const double nn = sqrt((nv[0] * nv[0] + nv[1] * nv[1]) + nv[2] * nv[2]);
        for (int a = 0; a < 3; ++a) N[3 * i + a] = nv[a] / nn;
    }
}

__global__ void k_sa_clear(int* flag) { *flag = 0; }

static bool sa_params_ok(const ad_params* p) {
    if (!p) return false;
    const double v[] = {p->a, p->ell, p->lambda, p->T};
    for (double x : v)
        if (!isfinite(x)) return false;
    return p->a > 0 && p->ell > 0 && p->T > 0;
}

static SaCoef sa_coef(const ad_params* p, double dt) {
    SaCoef k;
    const double w = 2.0 * kPi / p->T;
    const double lr = p->lambda / p->ell;
    k.ell = p->ell;
    k.cj = p->a * w * (9.0 / 64.0) * lr * lr;
    k.ck = w * (15.0 / 64.0) * (p->a / p->ell) * lr * lr;
    k.h2 = 0.5 * dt;
    k.dt = dt;
    k.dt6 = dt / 6.0;
    return k;
}

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace ad_sa

using namespace ad_sa;

extern "C" {

int ad_sa_workspace_size(int32_t S, uint64_t* bytes) {
    if (S < 1 || !bytes) return AD_EINVAL;
    /* flag, then YA, YB (R and N each), AR, AN */
    *bytes = 256 + 6 * align256((size_t)S * 3 * sizeof(double));
    return AD_OK;
}

int ad_sa_rhs(const ad_params* p, int32_t S, const double* R, const double* N, const double* phi, double* dR,
              double* dN, void* stream) {
    if (!sa_params_ok(p) || S < 1 || !R || !N || !phi || !dR || !dN) return AD_EINVAL;
    const SaCoef k = sa_coef(p, 1.0);
    hipLaunchKernelGGL(k_sa_rhs, dim3(S), dim3(SA_WG), 0, (hipStream_t)stream, k, S, R, N,
                       phi, dR, dN, (int*)nullptr);
    return hipGetLastError() == hipSuccess ? AD_OK : AD_EDEVICE;
}

int ad_sa_run(const ad_params* p, int32_t S, double* R, double* N, const double* phi, double dt, int64_t nsteps,
              void* workspace, uint64_t ws_bytes, void* stream) {
    if (!sa_params_ok(p) || S < 1 || !R || !N || !phi || !(dt > 0) || !isfinite(dt) || nsteps < 0 || !workspace)
        return AD_EINVAL;
    uint64_t need = 0;
    ad_sa_workspace_size(S, &need);
    if (ws_bytes < need || reinterpret_cast<uintptr_t>(workspace) % 256) return AD_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    char* b = static_cast<char*>(workspace);
    const size_t blk = align256((size_t)S * 3 * sizeof(double));
    int* flag = reinterpret_cast<int*>(b);
    double* YA_R = reinterpret_cast<double*>(b + 256);
    double* YA_N = reinterpret_cast<double*>(b + 256 + blk);
    double* YB_R = reinterpret_cast<double*>(b + 256 + 2 * blk);
    double* YB_N = reinterpret_cast<double*>(b + 256 + 3 * blk);
    double* AR = reinterpret_cast<double*>(b + 256 + 4 * blk);
    double* AN = reinterpret_cast<double*>(b + 256 + 5 * blk);
    const SaCoef k = sa_coef(p, dt);
    const dim3 grid(S), block(SA_WG); /* one work-group (one wave) per dumbbell */
    hipLaunchKernelGGL(k_sa_clear, dim3(1), dim3(1), 0, st, flag);
    for (int64_t n = 0; n < nsteps; ++n) {
        /* stage inputs: state, YA, YB, YA; outputs: YA, YB, YA, state */
        hipLaunchKernelGGL(k_sa_stage, grid, block, 0, st, k, S, 0, R, N, phi, R, N, YA_R, YA_N, AR, AN, flag);
        hipLaunchKernelGGL(k_sa_stage, grid, block, 0, st, k, S, 1, R, N, phi, YA_R, YA_N, YB_R, YB_N, AR, AN, flag);
        hipLaunchKernelGGL(k_sa_stage, grid, block, 0, st, k, S, 2, R, N, phi, YB_R, YB_N, YA_R, YA_N, AR, AN, flag);
        hipLaunchKernelGGL(k_sa_stage, grid, block, 0, st, k, S, 3, R, N, phi, YA_R, YA_N, YB_R, YB_N, AR, AN, flag);
        if (hipGetLastError() != hipSuccess) return AD_EDEVICE;
    }
    int h = 0;
    if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return AD_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return AD_EDEVICE;
    return h ? AD_ENONFINITE : AD_OK;
}

}  // extern "C"
