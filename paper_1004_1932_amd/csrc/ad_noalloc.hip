/*
 * ad_mobility_apply_static: the mobility product u = M(X) F of one system
 * (the computation of ad_mobility_apply) for callers that cannot allocate
 * device memory. It needs no context and no workspace: the pack, the
 * self-and-partner velocities, the partial sums and the work list live in
 * the file-scope array `scratch` below, which the code object holds on every
 * device it is loaded on until the process ends.
 *
 * The host never names `scratch` in a launch or a copy: in host code the
 * name is only a stand-in for the device symbol. The device address comes
 * from hipGetSymbolAddress, taken once per device (with that device
 * current) at the first call on it and kept in scratch_ptr[device].
 *
 * Every call on one device shares that device's array and leaves its
 * contents behind; each call rewrites everything it reads (the control
 * block's flag, the tables and the work list first, then the pack and the
 * partial sums), so no state carries over. Calls that overlap on one device
 * (two streams, two threads) race on the array.
 */
#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>

#include <algorithm>
#include <mutex>

#include "../../include/ad.h"
#include "ad_internal.h"

using ad::Coef;
using ad::Dev;
using ad::Item;

namespace {
constexpr size_t kScratchBytes = size_t(16) << 20; /* 16 MiB per device */
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices]; /* device address of `scratch`, per device */

size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

/* Offsets of the regions inside the scratch array for one system of N
 * spheres in the given launch shape. */
struct StaticLayout {
    size_t ctl, U0, dsys, sys_off, sys_P, sys_pbase, items, fitems, pA, pB, pC, pD, part, total;
    int nIB, P, nitems, ncomp;
    int tw, nfitems; /* AD_FP64: targets per work-group of the pair sum and its work list */
};

StaticLayout static_layout(int prec, int rpy, int N, const ad::PairShape& sh, bool fp64_blocks) {
    StaticLayout L{};
    const int IB = sh.ipl * sh.wg / sh.wj;
    const int jc = sh.jchunk < N ? sh.jchunk : N;
    L.nIB = (N + IB - 1) / IB;
    L.P = (N + jc - 1) / jc;
    L.nitems = L.nIB * L.P;
    L.ncomp = (rpy && prec != ad::PREC_FP32C) ? 6 : 3;
    const bool f32 = prec == ad::PREC_FP32C;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = up256(o + bytes);
        return at;
    };
    const size_t n = (size_t)N;
    L.ctl = take(sizeof(ad::Ctl));
    L.U0 = take(3 * n * 8);
    L.dsys = take(n / 2 * 4);
    L.sys_off = take(2 * 4);
    L.sys_P = take(4);
    L.sys_pbase = take(8);
    L.items = take((size_t)L.nitems * sizeof(Item));
    L.tw = ad::f64w_targets(N);
    L.nfitems = prec == ad::PREC_FP64 && fp64_blocks ? (N + L.tw - 1) / L.tw : 0;
    L.fitems = take((size_t)L.nfitems * sizeof(Item));
    L.pA = take(f32 ? n * 16 : 0);
    L.pB = take(f32 ? n * 16 : 0);
    L.pC = take(f32 ? n * 8 : 0);
    L.pD = take(f32 ? 0 : 3 * n * 16);
    L.part = take((size_t)L.P * L.ncomp * n * 8);
    L.total = o;
    return L;
}

/* The control block's flag, the one-system tables and the work lists:
 * item q covers target block q % nIB against source chunk q / nIB; AD_FP64's
 * pair sum item q covers targets [q tw, q tw + tw) against every source. */
__global__ void k_static_tables(ad::Ctl* ctl, int* dsys, int* sys_off, int* sys_P, long long* sys_pbase,
                                Item* items, int N, int IB, int jc, int nIB, int nitems, Item* fitems, int tw,
                                int nfitems) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) {
        ctl->flag = 0;
        sys_off[0] = 0;
        sys_off[1] = N;
        sys_P[0] = (N + jc - 1) / jc;
        sys_pbase[0] = 0;
    }
    if (g < N / 2) dsys[g] = 0;
    if (g < nitems) {
        const int ch = g / nIB, ib = g - ch * nIB;
        Item it;
        it.sys = 0;
        it.i0 = ib * IB;
        it.ni = min(IB, N - it.i0);
        it.j0 = ch * jc;
        it.nj = min(jc, N - it.j0);
        it.c = ch;
        it.Nb = N;
        it.ioff = 0;
        items[g] = it;
    }
    if (g < nfitems) {
        Item it;
        it.sys = 0;
        it.i0 = g * tw;
        it.ni = min(tw, N - it.i0);
        it.j0 = 0;
        it.nj = N;
        it.c = 0;
        it.Nb = N;
        it.ioff = 0;
        fitems[g] = it;
    }
}

/* device address of this device's scratch array (set up at the first call) */
int scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return ad::thread_fail(AD_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return ad::thread_fail(AD_EDEVICE, "device %d is beyond the %d devices this library tracks", dev,
                               kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return ad::thread_fail(AD_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                                   hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return AD_OK;
}

}  // namespace

extern "C" int ad_mobility_apply_static(const ad_params* p, int32_t N, const double* X, const double* F,
                                        double* u, void* stream) {
    ad::thread_clear_error();
    if (!p || !X || !F || !u) return ad::thread_fail(AD_EINVAL, "null argument");
    if (N < 2 || (N & 1)) return ad::thread_fail(AD_EINVAL, "N must be even and >= 2 (got %d)", N);
    if (!isfinite(p->a) || !isfinite(p->eta) || !(p->a > 0) || !(p->eta > 0))
        return ad::thread_fail(AD_EINVAL, "a and eta must be finite and > 0");
    if (p->precision != AD_FP64 && p->precision != AD_FP64_TILED && p->precision != AD_FP32C)
        return ad::thread_fail(AD_EINVAL, "precision must be AD_FP64, AD_FP64_TILED or AD_FP32C (got %d)",
                               p->precision);
    if (p->tensor != AD_OSEEN && p->tensor != AD_RPY)
        return ad::thread_fail(AD_EINVAL, "unknown tensor %d", p->tensor);
    const int prec = p->precision == AD_FP32C        ? ad::PREC_FP32C
                     : p->precision == AD_FP64_TILED ? ad::PREC_FP64_TILED
                                                     : ad::PREC_FP64;
    const int rpy = p->tensor == AD_RPY ? 1 : 0;
    const ad::PairShape ps = ad::default_pair_shape(prec, 1, N);
    /* AD_FP64 sums in k_pairs_f64w over a list of target blocks; where that
     * list does not fit beside the rest, in k_pairs_f64 with one source
     * chunk (the same bits, slower) */
    StaticLayout L = static_layout(prec, rpy, N, ps, true);
    if (L.total > kScratchBytes && L.nfitems > 0) L = static_layout(prec, rpy, N, ps, false);
    if (L.total > kScratchBytes)
        return ad::thread_fail(AD_ENOMEM,
                               "N = %d needs %zu bytes of scratch, more than the %zu bytes the library holds per "
                               "device",
                               N, L.total, kScratchBytes);
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc != AD_OK) return rc;
    char* b = static_cast<char*>(base);

    Dev d{};
    d.ctl = reinterpret_cast<ad::Ctl*>(b + L.ctl);
    d.U0 = reinterpret_cast<double*>(b + L.U0);
    d.dsys = reinterpret_cast<const int*>(b + L.dsys);
    d.sys_off = reinterpret_cast<const int*>(b + L.sys_off);
    d.sys_P = reinterpret_cast<const int*>(b + L.sys_P);
    d.sys_pbase = reinterpret_cast<const long long*>(b + L.sys_pbase);
    d.items = reinterpret_cast<const Item*>(b + L.items);
    d.fitems = reinterpret_cast<const Item*>(b + L.fitems);
    d.nfitems = L.nfitems;
    if (prec == ad::PREC_FP32C) {
        d.pA = reinterpret_cast<float4*>(b + L.pA);
        d.pB = reinterpret_cast<float4*>(b + L.pB);
        d.pC = reinterpret_cast<float2*>(b + L.pC);
    } else {
        d.pD = reinterpret_cast<double2*>(b + L.pD);
    }
    d.part = reinterpret_cast<double*>(b + L.part);
    d.ring = 1;
    d.Ntot = N;
    d.Stot = N / 2;
    d.nsys = 1;
    d.nitems = L.nitems;
    d.ncomp = L.ncomp;

    ad::Epi e{};
    e.c = ad::make_coef(p);
    e.prec = prec;
    e.integ = 0;
    e.stage = 0;
    e.nst = 4;
    e.pack_next = 1;
    e.u_aos = u;

    ad::Shape sh{};
    sh.wg = ps.wg;
    sh.wj = ps.wj;
    sh.ipl = ps.ipl;
    sh.split = prec == ad::PREC_FP32C ? 1 : 0; /* hi/lo positions, the default */
    sh.fused = 0;
    sh.rpy = rpy;
    sh.steric = 0;

    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int IB = ps.ipl * ps.wg / ps.wj;
    const int jc = ps.jchunk < N ? ps.jchunk : N;
    const int nthr = std::max(N, std::max(L.nitems, L.nfitems));
    hipLaunchKernelGGL(k_static_tables, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, st, d.ctl,
                       const_cast<int*>(d.dsys), const_cast<int*>(d.sys_off), const_cast<int*>(d.sys_P),
                       const_cast<long long*>(d.sys_pbase), const_cast<Item*>(d.items), N, IB, jc, L.nIB,
                       L.nitems, const_cast<Item*>(d.fitems), L.tw, L.nfitems);
    hipError_t err = hipGetLastError();
    if (err == hipSuccess) err = ad::launch_pack_apply(d, e.c, prec, X, F, st);
    if (err == hipSuccess) err = ad::launch_pairs(d, e, sh, 0, st);
    if (err == hipSuccess) err = ad::launch_epilogue(d, e, st);
    if (err != hipSuccess)
        return ad::thread_fail(AD_EDEVICE, "kernel launch failed: %s", hipGetErrorString(err));
    return AD_OK;
}
