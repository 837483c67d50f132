// Kernel templates: one workgroup per frame. The per-frame "hot" arena (PCG vectors,
// triangular-set search state, level lists) sits in LDS when it fits and in the frame's
// global workspace otherwise; HOT_LDS selects the placement at compile time so that the
// compiler emits LDS instructions for the LDS instantiation. Each combination of PCG
// precision and arena placement is instantiated in a translation unit of its own
// (lpdec_inst_*.hip), so that the four compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "lpdec_device.hpp"
#include "lpdec_launch.hpp"

namespace lpdec {


// A batch larger than the device holds at once: the grid is one resident set of workgroups,
// and each takes the next frame from a counter as it finishes one. Left to the hardware, the
// workgroups of a larger grid are dispatched strictly in index order, workgroup b to XCD
// b mod 8, so a compute unit that frees up waits until the next workgroup in line finds room on
// its own XCD. Measured on the n=1024 batch, compute units idled a median 9.5 ms (at most
// 185 ms) between frames.
template <typename PT>
LPD_INLINE void run_decode_claimed(Frame<PT> &F, const Args &a)
{
    for (;;) {
        __syncthreads();   // the previous frame's last reads of the scratch area are done
        if (F.tid == 0) F.sc->i[2] = __hip_atomic_fetch_add(a.next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int k = F.sc->i[2];
        __syncthreads();
        if (k >= a.nframes) return;
        F.decode(a, a.order ? a.order[k] : k);
    }
}

template <typename PT>
LPD_INLINE void run_ipm(Frame<PT> &F, const Args &a, int f)
{
    const int m = F.m, n = F.n;
    F.load_gamma(a, f);
    for (int j = F.tid; j < m; j += F.nt) F.vmask[j] = a.vmask_in[(size_t)f * m + j];
    __syncthreads();
    F.build_lists();
    lpdec_stats st = {};
    int its = 0;
    const int status = F.ipm(st, its);
    const size_t q = (size_t)n + m;
    for (int c = F.tid; c < n + m; c += F.nt) {
        const bool pr = F.colpresent(c);
        a.x_out[f * q + c] = pr ? F.x[c] : 0.0;
        a.z_out[f * q + c] = pr ? F.z[c] : 0.0;
    }
    for (int j = F.tid; j < m; j += F.nt) a.vec_out[(size_t)f * m + j] = F.cut(j) ? F.y[j] : 0.0;
    if (F.tid == 0) {
        a.i_out[f] = its;
        a.i_out2[f] = status;
        if (a.stats) { st.status = status; st.ipm_iters = its; a.stats[f] = st; }
    }
}

template <typename PT>
LPD_INLINE void run_solve(Frame<PT> &F, const Args &a, int f)
{
    const int m = F.m, n = F.n;
    const size_t q = (size_t)n + m;
    F.load_gamma(a, f);
    for (int j = F.tid; j < m; j += F.nt) {
        F.vmask[j] = a.vmask_in[(size_t)f * m + j];
        F.w[j] = a.vec_in[(size_t)f * m + j];
    }
    for (int c = F.tid; c < n + m; c += F.nt) {
        const double dd = a.d2_in[f * q + c];
        F.d2[c] = dd;
        F.set_d2f(c, dd);
    }
    __syncthreads();
    F.build_lists();
    F.find_precond_set();
    F.build_levels();
    int refr = 0, escal = 0;
    double resid2 = 0.0;
    bool met;
    const int its = F.solve(0.0, refr, escal, resid2, met);
    for (int j = F.tid; j < m; j += F.nt) a.vec_out[(size_t)f * m + j] = F.cut(j) ? F.dy[j] : 0.0;
    if (F.tid == 0) {
        if (a.i_out) a.i_out[f] = its;
        if (a.d_out) a.d_out[f] = sqrt(resid2);
    }
}

template <typename PT>
LPD_INLINE void run_matvec(Frame<PT> &F, const Args &a, int f)
{
    const int m = F.m, n = F.n;
    const size_t q = (size_t)n + m;
    F.load_gamma(a, f);
    for (int j = F.tid; j < m; j += F.nt) {
        F.vmask[j] = a.vmask_in[(size_t)f * m + j];
        F.h[j] = (PT)a.vec_in[(size_t)f * m + j];
    }
    for (int c = F.tid; c < n + m; c += F.nt) F.d2f[c] = (PT)a.d2_in[f * q + c];
    __syncthreads();
    F.build_lists();
    for (int i = F.tid; i < n; i += F.nt) F.t[i] = F.d2f[i] * F.template col_dot<PT>(i, F.h);
    for (int j = F.tid; j < m; j += F.nt) F.t[n + j] = F.d2f[n + j] * F.h[j];
    __syncthreads();
    for (int j = F.tid; j < m; j += F.nt)
        a.vec_out[(size_t)f * m + j] = F.cut(j) ? (double)F.template row_dot<PT>(j, F.t) : 0.0;
}

template <typename PT>
LPD_INLINE void run_mts(Frame<PT> &F, const Args &a, int f)
{
    const int m = F.m, n = F.n;
    for (int j = F.tid; j < m; j += F.nt) F.vmask[j] = a.hascut_in[(size_t)f * m + j] ? 1u : 0u;
    for (int i = F.tid; i < n; i += F.nt) F.sg[i] = 1;
    __syncthreads();
    F.build_lists();
    int rounds = 0;
    if (a.o.precond == 2 || a.o.precond == 3) F.mts_row(a.w_in + (size_t)f * (n + m), a.o.precond - 2);
    else if (a.o.precond == 5) F.mts_inc(a.w_in + (size_t)f * (n + m), rounds);
    else rounds = F.mts(a.w_in + (size_t)f * (n + m));
    for (int j = F.tid; j < m; j += F.nt) {
        a.i_out[(size_t)f * m + j] = F.pair[j];
        a.i_out2[(size_t)f * m + j] = F.lbv[j];
        a.i_out3[(size_t)f * m + j] = F.lfv[j];
    }
    if (F.tid == 0 && a.flag) a.flag[f] = a.o.precond == 5 ? rounds : F.p;
}

template <typename PT>
LPD_INLINE void run_cuts(Frame<PT> &F, const Args &a, int f)
{
    const int m = F.m, n = F.n;
    for (int i = F.tid; i < n; i += F.nt) F.u[i] = a.vec_in[(size_t)f * n + i];
    __syncthreads();
    for (int j = F.tid; j < m; j += F.nt) {
        uint32_t V;
        double lhs;
        const int vv = F.find_cut(j, V, lhs);
        a.u32_out[(size_t)f * m + j] = V;
        a.u8_out[(size_t)f * m + j] = (uint8_t)vv;
        if (a.vec_out) a.vec_out[(size_t)f * m + j] = lhs;
    }
}

// Persistent serving loop: thread 0 claims the next published ticket (compare-and-swap on a
// device counter, so every ticket is decoded exactly once and only after the host published
// it), the workgroup decodes that ring slot, and repeats. Without a ticket it sleeps and polls.
// The launch ends as a whole: once a workgroup has polled idle_polls times in a row while no
// workgroup held a ticket and none was unclaimed, it closes the launch and every workgroup
// leaves, so
// that a launch never goes on with only a few of its workgroups while requests come in.
// Between frames a workgroup also leaves when the host sets stop, or lowers the engine's share
// of workgroups below its index (so that another code's engine gets the compute unit). Tickets
// published after the launch closed stay unclaimed for the next launch.
template <typename PT>
LPD_INLINE void run_serve(Frame<PT> &F, const Args &a)
{
    int32_t *const busy = a.claim + 1, *const closing = a.claim + 2;
    constexpr int R = __ATOMIC_RELAXED;
    constexpr int AG = __HIP_MEMORY_SCOPE_AGENT, SY = __HIP_MEMORY_SCOPE_SYSTEM;
    for (;;) {
        __syncthreads();   // the previous frame's last reads of the scratch area are done
        if (F.tid == 0) {
            int got = -1;
            for (int polls = 0;; ++polls) {
                // relaxed polls: a system-scope acquire invalidates caches, and hundreds of
                // idle workgroups doing so every poll slow down the ones that decode; the one
                // acquire is taken after a successful claim
                if (__hip_atomic_load(a.stop, R, SY) || __hip_atomic_load(closing, R, AG)) break;
                if ((int)blockIdx.x >= __hip_atomic_load(a.share, R, SY)) break;
                const int pub = __hip_atomic_load(a.published, R, SY);
                int c = __hip_atomic_load(a.claim, R, AG);
                if (c < pub) {
                    // counted as busy before the claim, so that no workgroup closes the launch
                    // between this claim and its frame
                    __hip_atomic_fetch_add(busy, 1, R, AG);
                    if (__hip_atomic_compare_exchange_strong(a.claim, &c, c + 1, R, R, AG)) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");   // the slot's LLRs
                        got = c;
                        break;
                    }
                    __hip_atomic_fetch_add(busy, -1, R, AG);
                    continue;
                }
                // idle_polls polls in a row with no workgroup holding a ticket
                if (__hip_atomic_load(busy, R, AG) != 0) {
                    polls = -1;
                } else if (polls >= a.idle_polls) {
                    int zero = 0;
                    (void)__hip_atomic_compare_exchange_strong(closing, &zero, 1, R, R, AG);
                    break;
                }
                // 16 x 127 x 64 clocks (about 54 us at 2.4 GHz) between polls of the
                // host-mapped counter
                for (int k = 0; k < 16; ++k) __builtin_amdgcn_s_sleep(127);
            }
            F.sc->i[2] = got;
        }
        __syncthreads();
        const int t = F.sc->i[2];
        __syncthreads();
        if (t < 0) return;
        F.decode(a, t % a.ring);
        if (F.tid == 0) __hip_atomic_fetch_add(busy, -1, R, AG);
    }
}

template <typename PT, bool HOT_LDS, int MODE>
__global__ void __launch_bounds__(256) lpdec_main(Args a)
{
    extern __shared__ __align__(16) char lds_dyn[];
    __shared__ Scratch sc;
    const int f = blockIdx.x;
    if (f >= a.nframes) return;
    char *hot = HOT_LDS ? lds_dyn : a.hot_ws + (size_t)f * a.hot_stride;
    char *cold = a.cold_ws + (size_t)f * a.cold_stride;
    Frame<PT> F;
    // MODE_IPM may give every frame its own matrix (ALP: one LP row per cut)
    F.bind(a, a.codes ? a.codes[f] : a.code, hot, cold, &sc);
    // tiles of the dense fallback follow the hot arena in dynamic LDS
    F.ldsd = a.plan.dense_on ? (double *)(lds_dyn + (HOT_LDS ? lp_align(a.plan.hot_bytes) : 0)) : nullptr;
    if constexpr (MODE == MODE_DECODE) {
        if (a.next) run_decode_claimed(F, a);
        else F.decode(a, f);
    }
    else if constexpr (MODE == MODE_IPM) run_ipm(F, a, f);
    else if constexpr (MODE == MODE_SOLVE) run_solve(F, a, f);
    else if constexpr (MODE == MODE_MATVEC) run_matvec(F, a, f);
    else if constexpr (MODE == MODE_MTS) run_mts(F, a, f);
    else if constexpr (MODE == MODE_CUTS) run_cuts(F, a, f);
    else if constexpr (MODE == MODE_SERVE) run_serve(F, a);
}

template <typename PT, bool HOT_LDS, int MODE>
hipError_t launch_t(const Args &a, int block, size_t lds_bytes, hipStream_t stream, int grid)
{
    // the per-thread error state is shared with every other HIP user of the thread: drop an
    // unread error left by an earlier call so that only this launch is checked below
    (void)hipGetLastError();
    if (lds_bytes > 0) {
        // raises the dynamic-LDS limit of this kernel to what the hot arena and the dense
        // fallback's tiles need
        const hipError_t e = hipFuncSetAttribute((const void *)lpdec_main<PT, HOT_LDS, MODE>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((lpdec_main<PT, HOT_LDS, MODE>), dim3(grid), dim3(block), lds_bytes, stream, a);
    return hipGetLastError();
}

template <typename PT, bool HOT_LDS>
hipError_t launch_m(const Args &a, int block, size_t lds_bytes, hipStream_t stream, int grid)
{
    switch (a.mode) {
    case MODE_DECODE: return launch_t<PT, HOT_LDS, MODE_DECODE>(a, block, lds_bytes, stream, grid);
    case MODE_IPM: return launch_t<PT, HOT_LDS, MODE_IPM>(a, block, lds_bytes, stream, grid);
    case MODE_SOLVE: return launch_t<PT, HOT_LDS, MODE_SOLVE>(a, block, lds_bytes, stream, grid);
    case MODE_MATVEC: return launch_t<PT, HOT_LDS, MODE_MATVEC>(a, block, lds_bytes, stream, grid);
    case MODE_MTS: return launch_t<PT, HOT_LDS, MODE_MTS>(a, block, lds_bytes, stream, grid);
    case MODE_CUTS: return launch_t<PT, HOT_LDS, MODE_CUTS>(a, block, lds_bytes, stream, grid);
    case MODE_SERVE: return launch_t<PT, HOT_LDS, MODE_SERVE>(a, block, lds_bytes, stream, grid);
    default: return hipErrorInvalidValue;
    }
}

// Defines the launcher and the decode kernel's address of one instantiation.
#define LPDEC_INSTANTIATE(NAME, PT, HOT)                                                            \
    hipError_t launch_##NAME(const Args &a, int block, size_t lds, hipStream_t s, int grid)       \
    {                                                                                             \
        return launch_m<PT, HOT>(a, block, lds, s, grid);                                         \
    }                                                                                             \
    const void *decode_kernel_##NAME() { return (const void *)lpdec_main<PT, HOT, MODE_DECODE>; }

}  // namespace lpdec
