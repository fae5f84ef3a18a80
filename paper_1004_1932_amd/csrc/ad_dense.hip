/*
 * Dense baseline (AD_FP64_DENSE): every system's full 3Nb x 3Nb pair tensor
 * is assembled in HBM and then multiplied by the forces. This is the design
 * the paper used for its GPU code (Sec. V), kept as an ablation beside the
 * matrix-free pair sums: both kernels stream 72 Nb^2 bytes per stage, so the
 * stage is HBM bound instead of ALU bound. FP64 throughout.
 */
#include <hip/hip_ext.h>

#include "ad_internal.h"

namespace ad {

constexpr int DA_T = 256; /* target spheres per assembly work-group */
constexpr int DG_T = DENSE_ROWS; /* tensor rows per product work-group */
constexpr int DG_U = 32;  /* tensor loads in flight per thread (8: 11 % slower at N = 512) */

/* Block (i, j) of system b, i != j, r = X_i - X_j, rr = r r^T / r^2:
 *   T = (I + rr) / r                         Oseen (Eq. e:Mazur, first line)
 *     + (2a^2/3) (I - 3 rr) / r^3            RPY-Mazur correction (second line)
 * without the factor 1/(8 pi eta), which the epilogue applies after the
 * product. The (i, i) block is zero: the self term 1/(6 pi eta a) F_i is the
 * epilogue's u0. A coincident pair gives a zero block and raises the flag, as
 * in the pair sums. Element (3i+a, 3j+c) is stored column-major at
 * H[hbase_b + (3j+c) 3Nb + 3i+a], so a wave writes three contiguous runs.
 * Grid: x = source sphere (global), y = block of DA_T target spheres. */
__global__ __launch_bounds__(DA_T) void k_dense_assemble(Dev d, Epi e, int mode) {
    if (mode) advance_slots(d, e);
    const int J = blockIdx.x;
    const int b = d.dsys[J >> 1];
    const int off = d.sys_off[b];
    const int Nb = d.sys_off[b + 1] - off;
    const int il = blockIdx.y * DA_T + threadIdx.x;
    if (il >= Nb) return;
    const int jl = J - off;
    const int I = off + il;
    const double2 pi0 = d.pD[3 * I], pi1 = d.pD[3 * I + 1];
    const double2 pj0 = d.pD[3 * J], pj1 = d.pD[3 * J + 1];
    const double r[3] = {pi0.x - pj0.x, pi0.y - pj0.y, pi1.x - pj1.x};
    const double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    double T[3][3];
    if (il == jl || r2 == 0.0) {
        if (il != jl) atomicOr(&d.ctl->flag, FLAG_NONFINITE);
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) T[a][c] = 0.0;
    } else {
        const double ir = 1.0 / sqrt(r2);
        const double q = 1.0 / r2;
        const double w = e.c.rpy ? (e.c.cr / e.c.co) * (ir * q) : 0.0;
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                const double delta = a == c ? 1.0 : 0.0;
                const double rr = (r[a] * q) * r[c];
                double t = ir * (delta + rr);
                if (e.c.rpy) t = t + w * (delta - 3.0 * rr);
                T[a][c] = t;
            }
    }
    const long long ld = 3LL * Nb;
    double* H = d.H + d.sys_hbase[b] + 3LL * il;
    for (int c = 0; c < 3; ++c) {
        double* col = H + (3LL * jl + c) * ld;
        col[0] = T[0][c];
        col[1] = T[1][c];
        col[2] = T[2][c];
    }
}

/* Partial product of one work item: rows [i0, i0+ni) of system `sys`'s
 * tensor (local row 3i+a) against the columns of source spheres
 * [j0, j0+nj), the forces staged in LDS from the pack. One thread per row
 * sums its columns in ascending order (no FMA) into partial slot c, which the
 * epilogue adds over the chunks in order. Loads of a column are contiguous
 * across the wave. */
__global__ __launch_bounds__(DG_T) void k_dense_gemv(Dev d) {
    __shared__ double Fs[3 * DENSE_JMAX];
    const Item it = d.items[blockIdx.x];
    for (int q = threadIdx.x; q < it.nj; q += DG_T) {
        const int J = it.j0 + q;
        const double2 p1 = d.pD[3 * J + 1], p2 = d.pD[3 * J + 2];
        Fs[3 * q] = p1.y;
        Fs[3 * q + 1] = p2.x;
        Fs[3 * q + 2] = p2.y;
    }
    __syncthreads();
    const int row = it.i0 + (int)threadIdx.x;
    if (row >= it.i0 + it.ni) return;
    const int nc = 3 * it.nj;
    const long long ld = 3LL * it.Nb;
    const double* col = d.H + d.sys_hbase[it.sys] + 3LL * (it.j0 - it.ioff) * ld + row;
    double acc = 0.0;
    int c = 0;
    for (; c + DG_U <= nc; c += DG_U) {
        double h[DG_U];
#pragma unroll
        for (int u = 0; u < DG_U; ++u) h[u] = col[(long long)(c + u) * ld];
#pragma unroll
        for (int u = 0; u < DG_U; ++u) acc = acc + h[u] * Fs[c + u];
    }
    for (; c < nc; ++c) acc = acc + col[(long long)c * ld] * Fs[c];
    const int i = row / 3, a = row - 3 * i;
    d.part[d.sys_pbase[it.sys] + (long long)it.c * 3 * it.Nb + (long long)a * it.Nb + i] = acc;
}

hipError_t launch_dense(const Dev& d, const Epi& e, int mode, int maxNb, hipStream_t s, hipEvent_t ev_start,
                        hipEvent_t ev_stop) {
    if (d.nitems <= 0 || maxNb <= 0) return hipSuccess;
    const dim3 ga(d.Ntot, (maxNb + DA_T - 1) / DA_T);
    if (ev_start)
        hipExtLaunchKernelGGL(k_dense_assemble, ga, dim3(DA_T), 0, s, ev_start, nullptr, 0, d, e, mode);
    else
        hipLaunchKernelGGL(k_dense_assemble, ga, dim3(DA_T), 0, s, d, e, mode);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (ev_stop)
        hipExtLaunchKernelGGL(k_dense_gemv, dim3(d.nitems), dim3(DG_T), 0, s, nullptr, ev_stop, 0, d);
    else
        hipLaunchKernelGGL(k_dense_gemv, dim3(d.nitems), dim3(DG_T), 0, s, d);
    return hipGetLastError();
}

}  // namespace ad
