// Host side of the C ABI declared in include/lpdec.h: contexts, codes, options, device
// workspaces, launches, and the continuous-batching server.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lpdec_common.hpp"
#include "lpdec_launch.hpp"

using lpdec::Args;
using lpdec::Plan;

namespace {

struct Workspace {
    char *ptr = nullptr;
    size_t bytes = 0;
    bool fixed = false;   // a region the library may not grow (the allocation-free entry point)
};

hipError_t ws_ensure(Workspace &w, size_t bytes)
{
    if (bytes <= w.bytes) return hipSuccess;
    if (w.fixed) return hipErrorOutOfMemory;
    if (w.ptr) {
        hipError_t e = hipFree(w.ptr);
        if (e != hipSuccess) return e;
        w.ptr = nullptr;
        w.bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    hipError_t e = hipMalloc((void **)&w.ptr, want);
    if (e != hipSuccess) { w.ptr = nullptr; return e; }
    w.bytes = want;
    return hipSuccess;
}

void ws_free(Workspace &w)
{
    if (w.ptr) (void)hipFree(w.ptr);
    w.ptr = nullptr;
    w.bytes = 0;
}

}  // namespace

struct lpdec_ctx {
    int device = 0;
    lpdec::Opts opts{};
    int precision = -1;   // -1: per call default
    int block = 0;        // 0: automatic
    int server_streams = 8;
    int server_mode = 1;
    int lds_limit = 65536;
    int ncu = 256;        // compute units of the device
    int dispatch_order = 1;
    std::string err;
    Workspace ws;
    char *scratch = nullptr;   // the device's fixed region of lpdec_decode_batch_noalloc
};

struct lpdec_code {
    lpdec_ctx *ctx = nullptr;   // compared only: the context may be destroyed before the code
    int device = 0;             // the device holding the code's arrays
    int m = 0, n = 0, E = 0, dcmax = 0, dvmax = 0;
    int *d_rowptr = nullptr, *d_col = nullptr, *d_colptr = nullptr, *d_vlist = nullptr;
    std::vector<int> rowptr, col;
};

namespace {

lpdec_status fail(const lpdec_ctx *ctx, lpdec_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        const_cast<lpdec_ctx *>(ctx)->err = buf;
    }
    return st;
}

lpdec_status hipfail(const lpdec_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? LPDEC_ENOMEM : LPDEC_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

void default_opts(lpdec::Opts &o)
{
    o.malp_mode = 0;
    o.malp_max = 200;
    o.ipm_max = 100;
    o.pcg_maxit = 0;
    o.ref_max = 3;
    o.precond = 1;
    o.direct = 1;
    o.mts_reuse = 1;
    o.warm = 0;
    o.ipm_warm = 0.0;
    o.tau_viol = 1e-4;
    o.tau_act = 1e-4;
    o.tau_int = 1e-4;
    o.eps = 1e-8;
    o.eps_stall = 1e-7;
    o.tau_cost = 1e-8;
    o.sigma = 0.1;
    o.eta = 0.9995;
    o.pcg_tol = 1e-6;
    o.ref_tol = 1e-10;
    o.xi_tol = 0.9;
}

lpdec::CodeView view(const lpdec_code *c)
{
    lpdec::CodeView v;
    v.m = c->m; v.n = c->n; v.E = c->E; v.dcmax = c->dcmax; v.dvmax = c->dvmax;
    v.rowptr = c->d_rowptr; v.col = c->d_col; v.colptr = c->d_colptr; v.vlist = c->d_vlist;
    return v;
}

int auto_block(const lpdec_code *c)
{
    // one wave per frame for tiny codes, whose level sweeps have little work per level;
    // otherwise four: the column passes and the dense fallback's tile updates spread over
    // the waves, which outweighs the barriers between levels
    const int q = c->n + c->m;
    return q <= 600 ? 64 : 256;
}

// Fills the launch geometry and workspace of Args; launches one workgroup per frame.
lpdec_status launch(lpdec_ctx *ctx, const lpdec_code *code, Args &a, int pt64, Workspace &ws,
                    hipStream_t stream)
{
    if (a.nframes <= 0) return LPDEC_OK;
    a.code = view(code);
    a.o = ctx->opts;
    // the dense fallback exists only inside the IPM (decode and IPM modes)
    const bool dense = ctx->opts.direct && (a.mode == lpdec::MODE_DECODE || a.mode == lpdec::MODE_IPM ||
                                            a.mode == lpdec::MODE_SERVE);
    a.plan = lpdec::make_plan(code->m, code->n, code->dcmax, code->dvmax, pt64 ? 8 : 4, dense);
    const size_t lds_dense = a.plan.dense_on ? lpdec::kDenseLdsBytes : 0;
    const size_t lds_need = lpdec::lp_align(a.plan.hot_bytes) + lds_dense;
    const size_t lds_avail = (size_t)ctx->lds_limit - lpdec::static_lds_bytes() - 256;
    a.hot_in_lds = lds_need <= lds_avail;
    a.hot_stride = a.hot_in_lds ? 0 : lpdec::lp_align(a.plan.hot_bytes + 255) & ~(size_t)255;
    a.cold_stride = (a.plan.cold_bytes + 255) & ~(size_t)255;
    const size_t per = a.hot_stride + a.cold_stride;
    const int block = ctx->block > 0 ? ctx->block : auto_block(code);
    const size_t lds_launch = a.hot_in_lds ? lds_need : lds_dense;
    // a decode batch larger than the device holds at once runs as one resident set of
    // workgroups that take the frames in turn (hardest first with DISPATCH_ORDER 1); the
    // counter, order, weights and histogram follow the workgroups' arenas
    int grid = a.nframes;
    if (a.mode == lpdec::MODE_DECODE) {
        const long long cap = (long long)lpdec::decode_per_cu(pt64, a.hot_in_lds, block, lds_launch) * ctx->ncu;
        if (a.nframes > cap) grid = (int)cap;
    }
    const size_t nf4 = lpdec::lp_align(4 * (size_t)a.nframes);
    const size_t ord_full = 2 * nf4 + lpdec::lp_align(4 * ((size_t)code->m + 1));
    if (ws.fixed) {
        // a region that cannot grow holds as many arenas as fit beside the claim counter and
        // the ordering arrays; the rest of the frames are taken in turn
        if (a.mode != lpdec::MODE_DECODE) return fail(ctx, LPDEC_EINVAL, "fixed workspace is for decoding only");
        const size_t extra_max = ord_full + 256;
        const size_t fit = ws.bytes > extra_max ? (ws.bytes - extra_max) / per : 0;
        if (fit < 1)
            return fail(ctx, LPDEC_EINVAL, "one frame's workspace (%zu bytes) and the ordering arrays (%zu bytes) "
                        "exceed the fixed region of %zu bytes", per, extra_max, ws.bytes);
        if ((size_t)grid > fit) grid = (int)fit;
    }
    const bool claimed = grid < a.nframes;
    const bool ordered = claimed && ctx->dispatch_order;
    const size_t ord_bytes = ordered ? ord_full : 0;
    const size_t extra = ord_bytes + (claimed ? 256 : 0);
    hipError_t e = ws_ensure(ws, per * (size_t)grid + extra);
    if (e != hipSuccess) return hipfail(ctx, e, "workspace allocation");
    a.cold_ws = ws.ptr;
    a.hot_ws = ws.ptr + a.cold_stride * (size_t)grid;
    a.order = nullptr;
    a.next = nullptr;
    char *base = ws.ptr + per * (size_t)grid;
    if (ordered) {
        int32_t *order = (int32_t *)base, *w = (int32_t *)(base + nf4), *hist = (int32_t *)(base + 2 * nf4);
        e = lpdec::launch_order(a, order, w, hist, stream);
        if (e != hipSuccess) return hipfail(ctx, e, "order launch");
        a.order = order;
    }
    if (claimed) {
        a.next = (int32_t *)(base + ord_bytes);
        e = lpdec::launch_clear(a.next, 1, stream);
        if (e != hipSuccess) return hipfail(ctx, e, "counter clear");
    }
    e = lpdec::launch_main(a, pt64, block, lds_launch, stream, grid);
    if (e != hipSuccess) return hipfail(ctx, e, "kernel launch");
    return LPDEC_OK;
}

int precision_for(const lpdec_ctx *ctx, int call_default) { return ctx->precision >= 0 ? ctx->precision : call_default; }

lpdec_status check_common(lpdec_ctx *ctx, const lpdec_code *code, int nframes)
{
    if (!ctx) return LPDEC_EINVAL;
    if (!code || code->ctx != ctx) return fail(ctx, LPDEC_EINVAL, "code is null or belongs to another context");
    if (nframes < 0) return fail(ctx, LPDEC_EINVAL, "nframes < 0");
    ctx->err.clear();
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
    return LPDEC_OK;
}

}  // namespace

// ------------------------------------------------------------------------------ context
extern "C" lpdec_status lpdec_ctx_create(int device, lpdec_ctx **out)
{
    if (!out) return LPDEC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LPDEC_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return LPDEC_EDEVICE;
    auto *c = new (std::nothrow) lpdec_ctx();
    if (!c) return LPDEC_ENOMEM;
    c->device = device;
    default_opts(c->opts);
    int lds = 0, ncu = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->lds_limit = lds;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        c->ncu = ncu;
    // the device address of the allocation-free entry point's region (looked up once per
    // device); a failure here only disables that entry point
    if (lpdec::scratch_region(device, &c->scratch) != hipSuccess) {
        c->scratch = nullptr;
        (void)hipGetLastError();
    }
    *out = c;
    return LPDEC_OK;
}

extern "C" lpdec_status lpdec_ctx_destroy(lpdec_ctx *ctx)
{
    if (!ctx) return LPDEC_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ws_free(ctx->ws);
    delete ctx;
    return LPDEC_OK;
}

extern "C" const char *lpdec_last_error(const lpdec_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" lpdec_status lpdec_set_option(lpdec_ctx *ctx, int32_t key, double v)
{
    if (!ctx) return LPDEC_EINVAL;
    lpdec::Opts &o = ctx->opts;
    auto ipos = [&](int lo) { return v >= lo && v <= 1e9 && v == (double)(long long)v; };
    switch (key) {
    case LPDEC_OPT_MALP_MODE: if (v != 0 && v != 1) break; o.malp_mode = (int)v; return LPDEC_OK;
    case LPDEC_OPT_PRECISION: if (v != -1 && v != 0 && v != 1) break; ctx->precision = (int)v; return LPDEC_OK;
    case LPDEC_OPT_TAU_VIOL: if (!(v >= 0 && v < 1)) break; o.tau_viol = v; return LPDEC_OK;
    case LPDEC_OPT_TAU_ACT: if (!(v >= 0 && v < 1)) break; o.tau_act = v; return LPDEC_OK;
    case LPDEC_OPT_TAU_INT: if (!(v >= 0 && v < 0.5)) break; o.tau_int = v; return LPDEC_OK;
    case LPDEC_OPT_IPM_EPS: if (!(v > 0 && v < 1)) break; o.eps = v; return LPDEC_OK;
    case LPDEC_OPT_SIGMA: if (!(v > 0 && v < 1)) break; o.sigma = v; return LPDEC_OK;
    case LPDEC_OPT_ETA: if (!(v > 0 && v < 1)) break; o.eta = v; return LPDEC_OK;
    case LPDEC_OPT_PCG_TOL: if (!(v > 0 && v < 1)) break; o.pcg_tol = v; return LPDEC_OK;
    case LPDEC_OPT_PCG_MAXIT: if (!ipos(0)) break; o.pcg_maxit = (int)v; return LPDEC_OK;
    case LPDEC_OPT_REF_TOL: if (!(v > 0 && v < 1)) break; o.ref_tol = v; return LPDEC_OK;
    case LPDEC_OPT_REF_MAX: if (!ipos(0)) break; o.ref_max = (int)v; return LPDEC_OK;
    case LPDEC_OPT_IPM_MAX: if (!ipos(1)) break; o.ipm_max = (int)v; return LPDEC_OK;
    case LPDEC_OPT_MALP_MAX: if (!ipos(1)) break; o.malp_max = (int)v; return LPDEC_OK;
    case LPDEC_OPT_BLOCK:
        if (!(v == 0 || (ipos(64) && v <= 256 && ((int)v % 64) == 0))) break;
        ctx->block = (int)v;
        return LPDEC_OK;
    case LPDEC_OPT_PRECOND: if (!(ipos(0) && v <= 5)) break; o.precond = (int)v; return LPDEC_OK;
    case LPDEC_OPT_SERVER_STREAMS: if (!ipos(1) || v > 32) break; ctx->server_streams = (int)v; return LPDEC_OK;
    case LPDEC_OPT_SERVER_MODE: if (v != 0 && v != 1) break; ctx->server_mode = (int)v; return LPDEC_OK;
    case LPDEC_OPT_DISPATCH_ORDER: if (v != 0 && v != 1) break; ctx->dispatch_order = (int)v; return LPDEC_OK;
    case LPDEC_OPT_XI_TOL: if (!(v > 0 && v < 1)) break; o.xi_tol = v; return LPDEC_OK;
    case LPDEC_OPT_IPM_STALL: if (!(v >= 0 && v < 1)) break; o.eps_stall = v; return LPDEC_OK;
    case LPDEC_OPT_DIRECT_FALLBACK: if (v != 0 && v != 1) break; o.direct = (int)v; return LPDEC_OK;
    case LPDEC_OPT_MTS_REUSE: if (!ipos(1) || v > 1000) break; o.mts_reuse = (int)v; return LPDEC_OK;
    case LPDEC_OPT_WARM_START: if (v != 0 && v != 1) break; o.warm = (int)v; return LPDEC_OK;
    case LPDEC_OPT_IPM_WARM: if (!(v >= 0 && v <= 10)) break; o.ipm_warm = v; return LPDEC_OK;
    case LPDEC_OPT_TAU_COST: if (!(v >= 0 && v <= 1)) break; o.tau_cost = v; return LPDEC_OK;
    default: return fail(ctx, LPDEC_EINVAL, "unknown option key %d", key);
    }
    return fail(ctx, LPDEC_EINVAL, "bad value %g for option %d", v, key);
}

extern "C" lpdec_status lpdec_get_option(const lpdec_ctx *ctx, int32_t key, double *v)
{
    if (!ctx || !v) return LPDEC_EINVAL;
    const lpdec::Opts &o = ctx->opts;
    switch (key) {
    case LPDEC_OPT_MALP_MODE: *v = o.malp_mode; break;
    case LPDEC_OPT_PRECISION: *v = ctx->precision; break;
    case LPDEC_OPT_TAU_VIOL: *v = o.tau_viol; break;
    case LPDEC_OPT_TAU_ACT: *v = o.tau_act; break;
    case LPDEC_OPT_TAU_INT: *v = o.tau_int; break;
    case LPDEC_OPT_IPM_EPS: *v = o.eps; break;
    case LPDEC_OPT_SIGMA: *v = o.sigma; break;
    case LPDEC_OPT_ETA: *v = o.eta; break;
    case LPDEC_OPT_PCG_TOL: *v = o.pcg_tol; break;
    case LPDEC_OPT_PCG_MAXIT: *v = o.pcg_maxit; break;
    case LPDEC_OPT_REF_TOL: *v = o.ref_tol; break;
    case LPDEC_OPT_REF_MAX: *v = o.ref_max; break;
    case LPDEC_OPT_IPM_MAX: *v = o.ipm_max; break;
    case LPDEC_OPT_MALP_MAX: *v = o.malp_max; break;
    case LPDEC_OPT_BLOCK: *v = ctx->block; break;
    case LPDEC_OPT_PRECOND: *v = o.precond; break;
    case LPDEC_OPT_SERVER_STREAMS: *v = ctx->server_streams; break;
    case LPDEC_OPT_SERVER_MODE: *v = ctx->server_mode; break;
    case LPDEC_OPT_DISPATCH_ORDER: *v = ctx->dispatch_order; break;
    case LPDEC_OPT_XI_TOL: *v = o.xi_tol; break;
    case LPDEC_OPT_IPM_STALL: *v = o.eps_stall; break;
    case LPDEC_OPT_DIRECT_FALLBACK: *v = o.direct; break;
    case LPDEC_OPT_MTS_REUSE: *v = o.mts_reuse; break;
    case LPDEC_OPT_WARM_START: *v = o.warm; break;
    case LPDEC_OPT_IPM_WARM: *v = o.ipm_warm; break;
    case LPDEC_OPT_TAU_COST: *v = o.tau_cost; break;
    default: return LPDEC_EINVAL;
    }
    return LPDEC_OK;
}

// ------------------------------------------------------------------------------ code
extern "C" lpdec_status lpdec_code_create(lpdec_ctx *ctx, int32_t m, int32_t n, const int32_t *rowptr,
                                          const int32_t *col, lpdec_code **out)
{
    if (!ctx) return LPDEC_EINVAL;
    if (!out || !rowptr || !col) return fail(ctx, LPDEC_EINVAL, "null argument");
    *out = nullptr;
    if (m <= 0 || n <= 0 || m + n > 16383)
        return fail(ctx, LPDEC_EINVAL, "bad sizes m=%d n=%d (need m, n > 0 and m + n <= 16383)", m, n);
    if (rowptr[0] != 0) return fail(ctx, LPDEC_EINVAL, "rowptr[0] != 0");
    int dcmax = 0;
    for (int j = 0; j < m; ++j) {
        const int d = rowptr[j + 1] - rowptr[j];
        if (d < 1 || d > 15) return fail(ctx, LPDEC_EINVAL, "row %d has degree %d (need 1..15)", j, d);
        dcmax = std::max(dcmax, d);
        for (int e = rowptr[j]; e < rowptr[j + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n) return fail(ctx, LPDEC_EINVAL, "row %d: column %d out of range", j, col[e]);
            if (e > rowptr[j] && col[e] <= col[e - 1])
                return fail(ctx, LPDEC_EINVAL, "row %d: columns not strictly increasing", j);
        }
    }
    const int E = rowptr[m];
    auto *c = new (std::nothrow) lpdec_code();
    if (!c) return LPDEC_ENOMEM;
    c->ctx = ctx; c->device = ctx->device; c->m = m; c->n = n; c->E = E; c->dcmax = dcmax;
    c->rowptr.assign(rowptr, rowptr + m + 1);
    c->col.assign(col, col + E);
    std::vector<int> colptr(n + 1, 0), vlist(E);
    for (int e = 0; e < E; ++e) colptr[col[e] + 1]++;
    for (int i = 0; i < n; ++i) colptr[i + 1] += colptr[i];
    for (int i = 0; i < n; ++i) c->dvmax = std::max(c->dvmax, colptr[i + 1] - colptr[i]);
    if (c->dvmax > 16) {
        const int dv = c->dvmax;
        delete c;
        return fail(ctx, LPDEC_EINVAL, "a column has degree %d (need <= 16)", dv);
    }
    std::vector<int> fill(colptr.begin(), colptr.end() - 1);
    for (int j = 0; j < m; ++j)
        for (int e = rowptr[j]; e < rowptr[j + 1]; ++e) vlist[fill[col[e]]++] = (j << 5) | (e - rowptr[j]);
    hipError_t er = hipSetDevice(ctx->device);
    if (er == hipSuccess) er = hipMalloc((void **)&c->d_rowptr, sizeof(int) * (m + 1));
    if (er == hipSuccess) er = hipMalloc((void **)&c->d_col, sizeof(int) * E);
    if (er == hipSuccess) er = hipMalloc((void **)&c->d_colptr, sizeof(int) * (n + 1));
    if (er == hipSuccess) er = hipMalloc((void **)&c->d_vlist, sizeof(int) * E);
    if (er == hipSuccess) er = hipMemcpy(c->d_rowptr, rowptr, sizeof(int) * (m + 1), hipMemcpyHostToDevice);
    if (er == hipSuccess) er = hipMemcpy(c->d_col, col, sizeof(int) * E, hipMemcpyHostToDevice);
    if (er == hipSuccess) er = hipMemcpy(c->d_colptr, colptr.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice);
    if (er == hipSuccess) er = hipMemcpy(c->d_vlist, vlist.data(), sizeof(int) * E, hipMemcpyHostToDevice);
    if (er != hipSuccess) {
        lpdec_code_destroy(c);
        return hipfail(ctx, er, "code upload");
    }
    *out = c;
    return LPDEC_OK;
}

extern "C" lpdec_status lpdec_code_destroy(lpdec_code *c)
{
    if (!c) return LPDEC_EINVAL;
    (void)hipSetDevice(c->device);
    if (c->d_rowptr) (void)hipFree(c->d_rowptr);
    if (c->d_col) (void)hipFree(c->d_col);
    if (c->d_colptr) (void)hipFree(c->d_colptr);
    if (c->d_vlist) (void)hipFree(c->d_vlist);
    delete c;
    return LPDEC_OK;
}

// ------------------------------------------------------------------------------ decoding
static lpdec_status decode_batch_impl(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                      const void *gamma, int32_t gdt, uint8_t *xhat, int32_t *flag,
                                      double *obj, lpdec_stats *stats, double *u, uint32_t *trace,
                                      int32_t trace_cap, int pt64, Workspace &ws, hipStream_t stream,
                                      int32_t *done = nullptr)
{
    if (nframes > 0 && (!gamma || !xhat || !flag)) return fail(ctx, LPDEC_EINVAL, "null gamma/xhat/flag");
    if (gdt != 0 && gdt != 1) return fail(ctx, LPDEC_EINVAL, "gamma_dtype must be 0 (f32) or 1 (f64)");
    Args a{};
    a.nframes = nframes;
    a.mode = lpdec::MODE_DECODE;
    a.gamma = gamma;
    a.gamma_f64 = gdt;
    a.xhat = xhat; a.flag = flag; a.obj = obj; a.stats = stats; a.u_out = u;
    a.trace = trace; a.trace_cap = trace ? trace_cap : 0;
    a.done = done;
    return launch(ctx, code, a, pt64, ws, stream);
}

extern "C" lpdec_status lpdec_decode_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                           const void *gamma_dev, int32_t gamma_dtype, uint8_t *xhat_dev,
                                           int32_t *flag_dev, double *obj_dev, lpdec_stats *stats_dev,
                                           double *u_dev, void *stream)
{
    lpdec_status st = check_common(ctx, code, nframes);
    if (st) return st;
    return decode_batch_impl(ctx, code, nframes, gamma_dev, gamma_dtype, xhat_dev, flag_dev, obj_dev,
                             stats_dev, u_dev, nullptr, 0, precision_for(ctx, 1), ctx->ws, (hipStream_t)stream);
}

extern "C" lpdec_status lpdec_decode_batch_noalloc(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                                   const void *gamma_dev, int32_t gamma_dtype, uint8_t *xhat_dev,
                                                   int32_t *flag_dev, double *obj_dev, lpdec_stats *stats_dev,
                                                   double *u_dev, void *stream)
{
    lpdec_status st = check_common(ctx, code, nframes);
    if (st) return st;
    if (!ctx->scratch) return fail(ctx, LPDEC_EDEVICE, "the fixed device region was not found at context creation");
    Workspace fixed;
    fixed.ptr = ctx->scratch;
    fixed.bytes = lpdec::kScratchBytes;
    fixed.fixed = true;
    return decode_batch_impl(ctx, code, nframes, gamma_dev, gamma_dtype, xhat_dev, flag_dev, obj_dev,
                             stats_dev, u_dev, nullptr, 0, precision_for(ctx, 1), fixed, (hipStream_t)stream);
}

extern "C" lpdec_status lpdec_decode_batch_trace(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                                 const void *gamma_dev, int32_t gamma_dtype, uint8_t *xhat_dev,
                                                 int32_t *flag_dev, double *obj_dev, lpdec_stats *stats_dev,
                                                 double *u_dev, uint32_t *trace_dev, int32_t trace_cap)
{
    lpdec_status st = check_common(ctx, code, nframes);
    if (st) return st;
    if (!trace_dev || trace_cap <= 0) return fail(ctx, LPDEC_EINVAL, "trace buffer required");
    st = decode_batch_impl(ctx, code, nframes, gamma_dev, gamma_dtype, xhat_dev, flag_dev, obj_dev, stats_dev,
                           u_dev, trace_dev, trace_cap, precision_for(ctx, 1), ctx->ws, nullptr);
    if (st) return st;
    hipError_t e = hipDeviceSynchronize();
    return e == hipSuccess ? LPDEC_OK : hipfail(ctx, e, "decode");
}

extern "C" lpdec_status lpdec_decode(lpdec_ctx *ctx, const lpdec_code *code, const double *gamma, uint8_t *xhat,
                                     int32_t *flag, double *objective, lpdec_stats *stats, double *u)
{
    lpdec_status st = check_common(ctx, code, 1);
    if (st) return st;
    if (!gamma || !xhat || !flag) return fail(ctx, LPDEC_EINVAL, "null gamma/xhat/flag");
    const int n = code->n;
    // one device block holding gamma and every output of the frame
    struct Dev { double obj; lpdec_stats st; int32_t flag; };
    const size_t off_g = 0, off_u = lpdec::lp_align(8 * (size_t)n), off_x = off_u + lpdec::lp_align(8 * (size_t)n);
    const size_t off_d = off_x + lpdec::lp_align((size_t)n), total = off_d + sizeof(Dev);
    char *buf = nullptr;
    hipError_t e = hipMalloc((void **)&buf, total);
    if (e != hipSuccess) return hipfail(ctx, e, "hipMalloc");
    Dev *dv = (Dev *)(buf + off_d);
    e = hipMemcpy(buf + off_g, gamma, 8 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        st = decode_batch_impl(ctx, code, 1, buf + off_g, 1, (uint8_t *)(buf + off_x), &dv->flag, &dv->obj,
                               &dv->st, (double *)(buf + off_u), nullptr, 0, precision_for(ctx, 1), ctx->ws, nullptr);
        if (st) { (void)hipFree(buf); return st; }
        e = hipDeviceSynchronize();
    }
    Dev h;
    if (e == hipSuccess) e = hipMemcpy(xhat, buf + off_x, n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && u) e = hipMemcpy(u, buf + off_u, 8 * (size_t)n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&h, dv, sizeof(Dev), hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    if (e != hipSuccess) return hipfail(ctx, e, "decode");
    *flag = h.flag;
    if (objective) *objective = h.obj;
    if (stats) *stats = h.st;
    return LPDEC_OK;
}

// ------------------------------------------------------------------------------ steps
static lpdec_status run_sync(lpdec_ctx *ctx, const lpdec_code *code, Args &a, int pt64)
{
    lpdec_status st = launch(ctx, code, a, pt64, ctx->ws, nullptr);
    if (st) return st;
    hipError_t e = hipDeviceSynchronize();
    return e == hipSuccess ? LPDEC_OK : hipfail(ctx, e, "kernel");
}


// ------------------------------------------------------------------------------ ALP
namespace {

// A device buffer freed with its owner (host code of the ALP entry point only).
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    hipError_t get(size_t bytes)
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        return hipMalloc(&p, bytes ? bytes : 1);
    }
    template <typename T> T *as() const { return (T *)p; }
};

struct AlpFrame {
    std::vector<int> chk;        // check of every cut, in the order the cuts were added
    std::vector<uint32_t> V;     // odd set of every cut (bit k = k-th variable of the check)
    std::vector<double> u;       // the last LP solution (hard decisions before the first)
    double gneg = 0.0, cost_prev = 0.0;
    int status = 0;
    bool done = false;
    lpdec_stats st{};
};

}  // namespace

extern "C" lpdec_status lpdec_alp_decode_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                               const double *gamma, uint8_t *xhat, int32_t *flag,
                                               double *objective, lpdec_stats *stats, double *u_out)
{
    lpdec_status st = check_common(ctx, code, nframes);
    if (st) return st;
    if (nframes == 0) return LPDEC_OK;
    if (!gamma || !xhat || !flag) return fail(ctx, LPDEC_EINVAL, "null gamma/xhat/flag");
    const int m = code->m, n = code->n, nf = nframes;
    const lpdec::Opts &o = ctx->opts;
    const int pt64 = precision_for(ctx, 1);
    std::vector<AlpFrame> F(nf);
    for (int f = 0; f < nf; ++f) {
        F[f].u.resize(n);
        for (int i = 0; i < n; ++i) {
            const double g = gamma[(size_t)f * n + i];
            F[f].u[i] = g >= 0.0 ? 0.0 : 1.0;
            if (g < 0.0) F[f].gneg += g;
        }
        F[f].cost_prev = F[f].gneg;
    }
    DevBuf d_gamma, d_u, d_vm, d_viol, d_lhs;
    hipError_t e = d_gamma.get(8 * (size_t)nf * n);
    if (e == hipSuccess) e = d_u.get(8 * (size_t)nf * n);
    if (e == hipSuccess) e = d_vm.get(4 * (size_t)nf * m);
    if (e == hipSuccess) e = d_viol.get((size_t)nf * m);
    if (e == hipSuccess) e = d_lhs.get(8 * (size_t)nf * m);
    if (e != hipSuccess) return hipfail(ctx, e, "ALP buffers");
    std::vector<double> hu((size_t)nf * n), hg((size_t)nf * n);
    std::vector<uint32_t> hvm((size_t)nf * m);
    std::vector<uint8_t> hviol((size_t)nf * m);
    std::vector<int> act;
    for (int k = 0; k < o.malp_max; ++k) {
        act.clear();
        for (int f = 0; f < nf; ++f)
            if (!F[f].done) act.push_back(f);
        if (act.empty()) break;
        const int na = (int)act.size();
        // Algorithm 2 on every check at the last solution of every active frame
        for (int a = 0; a < na; ++a) std::memcpy(&hu[(size_t)a * n], F[act[a]].u.data(), 8 * (size_t)n);
        e = hipMemcpy(d_u.p, hu.data(), 8 * (size_t)na * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hipfail(ctx, e, "ALP upload");
        Args ac{};
        ac.nframes = na; ac.mode = lpdec::MODE_CUTS;
        ac.vec_in = d_u.as<double>(); ac.u32_out = d_vm.as<uint32_t>(); ac.u8_out = d_viol.as<uint8_t>();
        ac.vec_out = d_lhs.as<double>();
        st = run_sync(ctx, code, ac, 1);
        if (st) return st;
        e = hipMemcpy(hvm.data(), d_vm.p, 4 * (size_t)na * m, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(hviol.data(), d_viol.p, (size_t)na * m, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hipfail(ctx, e, "ALP cut search");
        // every violated inequality joins its frame's LP; no cut is ever removed
        std::vector<int> lp;   // frames with new cuts
        for (int a = 0; a < na; ++a) {
            AlpFrame &R = F[act[a]];
            bool added = false;
            for (int j = 0; j < m; ++j)
                if (hviol[(size_t)a * m + j]) {
                    R.chk.push_back(j);
                    R.V.push_back(hvm[(size_t)a * m + j]);
                    added = true;
                }
            if (added) lp.push_back(act[a]);
            else R.done = true;
        }
        if (lp.empty()) break;
        // a frame whose LP no longer fits the list encoding (a variable in more than 16 cuts,
        // or more than 16383 - n cuts) ends with LPDEC_FLAG_ALP_CAPACITY
        {
            std::vector<int> keep, cnt(n);
            for (int f : lp) {
                const AlpFrame &R = F[f];
                std::fill(cnt.begin(), cnt.end(), 0);
                int dv = 0;
                for (int j : R.chk)
                    for (int t = code->rowptr[j]; t < code->rowptr[j + 1]; ++t) dv = std::max(dv, ++cnt[code->col[t]]);
                if (dv > 16 || (int)R.chk.size() + n > 16383) {
                    F[f].status = LPDEC_FLAG_ALP_CAPACITY;
                    F[f].done = true;
                } else {
                    keep.push_back(f);
                }
            }
            lp.swap(keep);
        }
        if (lp.empty()) continue;
        // one matrix per frame: row r is the row of the check of cut r; empty rows pad every
        // frame to the largest cut count of the launch (they carry no cut, so the LP ignores them)
        const int nl = (int)lp.size();
        int M = 0;
        for (int f : lp) M = std::max(M, (int)F[f].chk.size());
        std::vector<std::vector<int>> rp(nl), cl(nl), cp(nl), vl(nl);
        int dvmax = 1;
        size_t words = 0;
        for (int b = 0; b < nl; ++b) {
            const AlpFrame &R = F[lp[b]];
            auto &rowp = rp[b], &colv = cl[b], &colp = cp[b], &vlst = vl[b];
            rowp.assign(M + 1, 0);
            for (int r = 0; r < (int)R.chk.size(); ++r) {
                const int j = R.chk[r];
                for (int t = code->rowptr[j]; t < code->rowptr[j + 1]; ++t) colv.push_back(code->col[t]);
                rowp[r + 1] = (int)colv.size();
            }
            for (int r = (int)R.chk.size(); r < M; ++r) rowp[r + 1] = (int)colv.size();
            const int E = (int)colv.size();
            colp.assign(n + 1, 0);
            for (int t = 0; t < E; ++t) colp[colv[t] + 1]++;
            for (int i = 0; i < n; ++i) {
                dvmax = std::max(dvmax, colp[i + 1]);
                colp[i + 1] += colp[i];
            }
            vlst.assign(E, 0);
            std::vector<int> fill(colp.begin(), colp.end() - 1);
            for (int r = 0; r < M; ++r)
                for (int t = rowp[r]; t < rowp[r + 1]; ++t) vlst[fill[colv[t]]++] = (r << 5) | (t - rowp[r]);
            words += (size_t)(M + 1) + E + (n + 1) + E;
        }
        std::vector<int> hcsr(words);
        std::vector<lpdec::CodeView> views(nl);
        std::vector<uint32_t> hmask((size_t)nl * M, 0u);
        DevBuf d_csr, d_views, d_mask, d_g, d_x, d_z, d_y, d_its, d_status, d_stats;
        e = d_csr.get(4 * words);
        if (e == hipSuccess) e = d_views.get(sizeof(lpdec::CodeView) * nl);
        if (e == hipSuccess) e = d_mask.get(4 * (size_t)nl * M);
        if (e == hipSuccess) e = d_g.get(8 * (size_t)nl * n);
        if (e == hipSuccess) e = d_x.get(8 * (size_t)nl * (n + M));
        if (e == hipSuccess) e = d_z.get(8 * (size_t)nl * (n + M));
        if (e == hipSuccess) e = d_y.get(8 * (size_t)nl * M);
        if (e == hipSuccess) e = d_its.get(4 * (size_t)nl);
        if (e == hipSuccess) e = d_status.get(4 * (size_t)nl);
        if (e == hipSuccess) e = d_stats.get(sizeof(lpdec_stats) * nl);
        if (e != hipSuccess) return hipfail(ctx, e, "ALP LP buffers");
        size_t w = 0;
        for (int b = 0; b < nl; ++b) {
            const AlpFrame &R = F[lp[b]];
            const int E = (int)cl[b].size();
            lpdec::CodeView &v = views[b];
            v.m = M; v.n = n; v.E = E; v.dcmax = code->dcmax; v.dvmax = dvmax;
            int *base = d_csr.as<int>() + w;
            std::memcpy(&hcsr[w], rp[b].data(), 4 * (size_t)(M + 1)); v.rowptr = base; w += M + 1; base += M + 1;
            std::memcpy(&hcsr[w], cl[b].data(), 4 * (size_t)E); v.col = base; w += E; base += E;
            std::memcpy(&hcsr[w], cp[b].data(), 4 * (size_t)(n + 1)); v.colptr = base; w += n + 1; base += n + 1;
            std::memcpy(&hcsr[w], vl[b].data(), 4 * (size_t)E); v.vlist = base; w += E;
            for (int r = 0; r < (int)R.V.size(); ++r) hmask[(size_t)b * M + r] = R.V[r];
            std::memcpy(&hg[(size_t)b * n], gamma + (size_t)lp[b] * n, 8 * (size_t)n);
        }
        e = hipMemcpy(d_csr.p, hcsr.data(), 4 * words, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_views.p, views.data(), sizeof(lpdec::CodeView) * nl, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_mask.p, hmask.data(), 4 * (size_t)nl * M, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_g.p, hg.data(), 8 * (size_t)nl * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hipfail(ctx, e, "ALP LP upload");
        // the launch is sized for the padded matrices (M rows, column degree dvmax)
        lpdec_code shape;
        shape.m = M; shape.n = n; shape.E = 0; shape.dcmax = code->dcmax; shape.dvmax = dvmax;
        Args ai{};
        ai.nframes = nl; ai.mode = lpdec::MODE_IPM; ai.codes = d_views.as<lpdec::CodeView>();
        ai.gamma = d_g.p; ai.gamma_f64 = 1; ai.vmask_in = d_mask.as<uint32_t>();
        ai.x_out = d_x.as<double>(); ai.z_out = d_z.as<double>(); ai.vec_out = d_y.as<double>();
        ai.i_out = d_its.as<int32_t>(); ai.i_out2 = d_status.as<int32_t>(); ai.stats = d_stats.as<lpdec_stats>();
        st = run_sync(ctx, &shape, ai, pt64);
        if (st) return st;
        std::vector<double> hx((size_t)nl * (n + M));
        std::vector<int32_t> hits(nl), hst(nl);
        std::vector<lpdec_stats> hs(nl);
        e = hipMemcpy(hx.data(), d_x.p, 8 * hx.size(), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(hits.data(), d_its.p, 4 * (size_t)nl, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(hst.data(), d_status.p, 4 * (size_t)nl, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(hs.data(), d_stats.p, sizeof(lpdec_stats) * nl, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hipfail(ctx, e, "ALP LP results");
        for (int b = 0; b < nl; ++b) {
            AlpFrame &R = F[lp[b]];
            const double *g = gamma + (size_t)lp[b] * n;
            const double *x = &hx[(size_t)b * (n + M)];
            R.st.malp_iters++;
            R.st.ipm_iters += hits[b];
            R.st.pcg_iters += hs[b].pcg_iters;
            R.st.ref_rounds += hs[b].ref_rounds;
            R.st.mts_rounds += hs[b].mts_rounds;
            R.st.escalations += hs[b].escalations;
            R.st.direct_solves += hs[b].direct_solves;
            R.st.max_levels = std::max(R.st.max_levels, hs[b].max_levels);
            R.st.pcg_rows += hs[b].pcg_rows;
            R.st.ipm_cols += hs[b].ipm_cols;
            R.st.ticks_mts += hs[b].ticks_mts;
            R.st.ticks_solve += hs[b].ticks_solve;
            R.st.ticks_pcg += hs[b].ticks_pcg;
            R.st.ticks_dense += hs[b].ticks_dense;
            R.st.dense_cube += hs[b].dense_cube;
            R.st.p_max = std::max(R.st.p_max, (int)R.chk.size());
            if (hst[b] < 0) { R.status = hst[b]; R.done = true; continue; }
            // u^k on the box (Theorem 2a), then the cost check (Theorem 2b), as in MALP
            double cost = 0.0;
            for (int i = 0; i < n; ++i) {
                const double ui = std::min(1.0, std::max(0.0, g[i] >= 0.0 ? x[i] : 1.0 - x[i]));
                R.u[i] = ui;
                cost += g[i] * ui;
            }
            if (cost < R.cost_prev - o.tau_cost * (1.0 + std::fabs(R.cost_prev - R.gneg))) {
                R.status = LPDEC_FLAG_COST_DECREASE;
                R.done = true;
                continue;
            }
            R.cost_prev = cost;
        }
    }
    // output: integrality, decisions, syndrome, certificate flag, objective
    for (int f = 0; f < nf; ++f) {
        AlpFrame &R = F[f];
        if (!R.done && R.status == 0) R.status = LPDEC_FLAG_MALP_CAP;
        const double *g = gamma + (size_t)f * n;
        uint8_t *xh = xhat + (size_t)f * n;
        double fr = 0.0, ob = 0.0;
        for (int i = 0; i < n; ++i) {
            const double ui = R.u[i];
            fr = std::max(fr, std::min(ui, 1.0 - ui));
            ob += g[i] * ui;
            xh[i] = std::fabs(ui - 0.5) <= o.tau_int ? (g[i] >= 0.0 ? 0 : 1) : (ui > 0.5 ? 1 : 0);
            if (u_out) u_out[(size_t)f * n + i] = ui;
        }
        int syn = 0;
        for (int j = 0; j < m; ++j) {
            int par = 0;
            for (int t = code->rowptr[j]; t < code->rowptr[j + 1]; ++t) par ^= xh[code->col[t]];
            syn |= par;
        }
        int fl;
        if (R.status < 0) fl = R.status;
        else if (fr <= o.tau_int && !syn) fl = 1;
        else if (fr <= o.tau_int) fl = LPDEC_FLAG_INCONSISTENT;
        else fl = 0;
        flag[f] = fl;
        if (objective) objective[f] = ob;
        R.st.status = R.status < 0 ? R.status : 0;
        if (stats) stats[f] = R.st;
    }
    return LPDEC_OK;
}

extern "C" lpdec_status lpdec_cut_search_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                               const double *u_dev, uint32_t *vmask_dev, uint8_t *viol_dev,
                                               double *lhs_dev)
{
    lpdec_status st = check_common(ctx, code, nframes);
    if (st) return st;
    if (nframes > 0 && (!u_dev || !vmask_dev || !viol_dev)) return fail(ctx, LPDEC_EINVAL, "null argument");
    Args a{};
    a.nframes = nframes; a.mode = lpdec::MODE_CUTS;
    a.vec_in = u_dev; a.u32_out = vmask_dev; a.u8_out = viol_dev; a.vec_out = lhs_dev;
    return run_sync(ctx, code, a, 1);
}

extern "C" lpdec_status lpdec_mts_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                        const uint8_t *hascut_dev, const float *w_dev, int32_t *pair_dev,
                                        int32_t *lev_b_dev, int32_t *lev_f_dev, int32_t *rounds_dev)
{
    lpdec_status st = check_common(ctx, code, nframes);
    if (st) return st;
    if (nframes > 0 && (!hascut_dev || !w_dev || !pair_dev || !lev_b_dev || !lev_f_dev))
        return fail(ctx, LPDEC_EINVAL, "null argument");
    Args a{};
    a.nframes = nframes; a.mode = lpdec::MODE_MTS;
    a.hascut_in = hascut_dev; a.w_in = w_dev;
    a.i_out = pair_dev; a.i_out2 = lev_b_dev; a.i_out3 = lev_f_dev; a.flag = rounds_dev;
    return run_sync(ctx, code, a, 0);
}

extern "C" lpdec_status lpdec_normal_matvec_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                                  const uint32_t *vmask_dev, const double *gamma_dev,
                                                  const double *d2_dev, const double *h_dev, double *l_dev,
                                                  int32_t precision)
{
    lpdec_status st = check_common(ctx, code, nframes);
    if (st) return st;
    if (nframes > 0 && (!vmask_dev || !gamma_dev || !d2_dev || !h_dev || !l_dev))
        return fail(ctx, LPDEC_EINVAL, "null argument");
    if (precision != 0 && precision != 1) return fail(ctx, LPDEC_EINVAL, "precision must be 0 or 1");
    Args a{};
    a.nframes = nframes; a.mode = lpdec::MODE_MATVEC;
    a.vmask_in = vmask_dev; a.gamma = gamma_dev; a.gamma_f64 = 1; a.d2_in = d2_dev; a.vec_in = h_dev;
    a.vec_out = l_dev;
    return run_sync(ctx, code, a, precision);
}

extern "C" lpdec_status lpdec_newton_solve_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                                 const uint32_t *vmask_dev, const double *gamma_dev,
                                                 const double *d2_dev, const double *w_dev, double *y_dev,
                                                 int32_t *iters_dev, double *resid_dev, int32_t precision)
{
    lpdec_status st = check_common(ctx, code, nframes);
    if (st) return st;
    if (nframes > 0 && (!vmask_dev || !gamma_dev || !d2_dev || !w_dev || !y_dev))
        return fail(ctx, LPDEC_EINVAL, "null argument");
    if (precision != 0 && precision != 1) return fail(ctx, LPDEC_EINVAL, "precision must be 0 or 1");
    Args a{};
    a.nframes = nframes; a.mode = lpdec::MODE_SOLVE;
    a.vmask_in = vmask_dev; a.gamma = gamma_dev; a.gamma_f64 = 1; a.d2_in = d2_dev; a.vec_in = w_dev;
    a.vec_out = y_dev; a.i_out = iters_dev; a.d_out = resid_dev;
    return run_sync(ctx, code, a, precision);
}

extern "C" lpdec_status lpdec_ipm_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                        const uint32_t *vmask_dev, const double *gamma_dev, double *x_dev,
                                        double *y_dev, double *z_dev, int32_t *iters_dev, int32_t *status_dev,
                                        int32_t precision)
{
    lpdec_status st = check_common(ctx, code, nframes);
    if (st) return st;
    if (nframes > 0 && (!vmask_dev || !gamma_dev || !x_dev || !y_dev || !z_dev || !iters_dev || !status_dev))
        return fail(ctx, LPDEC_EINVAL, "null argument");
    if (precision != 0 && precision != 1) return fail(ctx, LPDEC_EINVAL, "precision must be 0 or 1");
    Args a{};
    a.nframes = nframes; a.mode = lpdec::MODE_IPM;
    a.vmask_in = vmask_dev; a.gamma = gamma_dev; a.gamma_f64 = 1;
    a.x_out = x_dev; a.z_out = z_dev; a.vec_out = y_dev; a.i_out = iters_dev; a.i_out2 = status_dev;
    return run_sync(ctx, code, a, precision);
}

// ------------------------------------------------------------------------------ serving
// Continuous batching. Submitted frames wait in a host queue. A scheduler thread forms a
// wave whenever one of its streams is idle: the queue head and the later queued frames of
// the same code, while the wave's device footprint fits in the free part of the HBM budget and
// the slots in flight stay under max_slots, copies their gamma to the wave's device buffer,
// launches the decode kernel on that stream and records an event. Waves on different
// streams overlap on the device. Each frame's results go to host-mapped pinned memory with a
// done flag that the kernel raises once they are visible, so the scheduler hands a frame's
// result out as soon as that frame is decoded, not when its wave ends; a wave's memory and
// slots are released when its kernel ends, and frames that arrived meanwhile are admitted.
namespace {

struct Request {
    uint64_t ticket;
    const lpdec_code *code;
    std::vector<double> gamma;
    std::chrono::steady_clock::time_point t_submit;
};

struct Result {
    std::vector<uint8_t> xhat;
    int32_t flag = 0;
    double obj = 0.0;
    double latency = 0.0;
};

// Host-mapped pinned memory (fine-grained): the kernel writes a frame's results and its done
// flag here, and the server thread reads them while the wave still runs.
struct HostOut {
    char *h = nullptr;            // host address
    char *d = nullptr;            // the same memory as the device addresses it
    size_t bytes = 0;
};

hipError_t hostout_ensure(HostOut &o, size_t bytes)
{
    if (bytes <= o.bytes) return hipSuccess;
    if (o.h) {
        hipError_t e = hipHostFree(o.h);
        if (e != hipSuccess) return e;
        o.h = o.d = nullptr;
        o.bytes = 0;
    }
    const size_t want = bytes + bytes / 4;
    hipError_t e = hipHostMalloc((void **)&o.h, want, hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) { o.h = nullptr; return e; }
    e = hipHostGetDevicePointer((void **)&o.d, o.h, 0);
    if (e != hipSuccess) { (void)hipHostFree(o.h); o.h = o.d = nullptr; return e; }
    o.bytes = want;
    return hipSuccess;
}

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Workspace ws;                 // kernel workspace of the wave in flight (its admitted footprint)
    Workspace io;                 // gamma in
    HostOut out;                  // xhat | flag | obj | done of every frame of the wave
    std::vector<Request> wave;    // frames in flight on this lane
    std::vector<char> retired;    // per frame: its result has been taken
    int nretired = 0;
    size_t footprint = 0;
    bool busy = false;
};

// Persistent engine of one code (server mode 1): a kernel of W workgroups that claim tickets
// from a ring of R request slots in host-mapped memory, each slot holding the frame's LLRs and
// its results. Device ticket t uses slot t mod R; the host publishes t only once the slot's
// previous ticket has been retired.
struct Engine {
    const lpdec_code *code = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ended = nullptr;
    Workspace ws;                 // kernel workspace of the W workgroups
    int32_t *claim = nullptr;     // device: tickets claimed so far
    HostOut ring;                 // gamma | xhat | flag | obj | done per slot, then published,
                                  // stop, share
    int R = 0, W = 0;
    size_t off_x = 0, off_f = 0, off_o = 0, off_d = 0, off_c = 0;
    int32_t published = 0;        // tickets published (the host's copy of the ring counter)
    std::vector<Request> slot;    // the request each used slot holds
    std::vector<char> used;
    std::deque<Request> backlog;  // taken from the queue, waiting for their slot
    int outstanding = 0;          // published and not yet retired
    bool running = false;
    size_t footprint = 0;
    int32_t *ctl() const { return (int32_t *)(ring.h + off_c); }
};

}  // namespace

struct lpdec_server {
    lpdec_ctx *ctx = nullptr;
    size_t budget = 0;
    int max_slots = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::map<uint64_t, Result> results;
    std::map<uint64_t, int> pending;   // ticket -> 1 while queued or running
    uint64_t next_ticket = 1;
    std::vector<Lane> lanes;
    int mode = 0;                                  // 0: waves on streams; 1: persistent engines
    std::vector<std::unique_ptr<Engine>> engines;  // mode 1, owned by the server thread
    int ncu = 0;
    size_t in_use = 0;
    int slots_in_use = 0;
    bool stop = false;
    std::thread worker;
    std::string err;
};

namespace {

// A server lane's device memory: stream-ordered allocation on the lane's stream, freed on that
// stream when the wave retires, so that the memory held matches the admitted footprints.
hipError_t lane_alloc(Workspace &w, size_t bytes, hipStream_t stream)
{
    w.ptr = nullptr;
    w.bytes = 0;
    w.fixed = true;
    const hipError_t e = hipMallocAsync((void **)&w.ptr, bytes ? bytes : 1, stream);
    if (e == hipSuccess) w.bytes = bytes;
    else w.ptr = nullptr;
    return e;
}

void lane_release(Lane &L)
{
    if (L.ws.ptr) (void)hipFreeAsync(L.ws.ptr, L.stream);
    if (L.io.ptr) (void)hipFreeAsync(L.io.ptr, L.stream);
    L.ws = Workspace{};
    L.io = Workspace{};
}

size_t frame_footprint(const lpdec_code *c, int pt64)
{
    Plan p = lpdec::make_plan(c->m, c->n, c->dcmax, c->dvmax, pt64 ? 8 : 4, c->ctx->opts.direct != 0);
    // cold arena + hot arena (counted even when it lives in LDS) + gamma + outputs
    return p.cold_bytes + p.hot_bytes + 8 * (size_t)c->n + (size_t)c->n + 64;
}

void server_loop(lpdec_server *s)
{
    // Lane state belongs to this thread alone; the mutex guards what the client calls share
    // (queue, results, pending, budget counters), and no HIP call is made while holding it.
    (void)hipSetDevice(s->ctx->device);
    const int pt64 = precision_for(s->ctx, 1);
    while (true) {
        // retire finished frames as their done flags appear, and a lane once its kernel ended
        std::vector<std::pair<uint64_t, Result>> done;
        size_t freed_bytes = 0;
        int freed_slots = 0;
        for (auto &L : s->lanes) {
            if (!L.busy) continue;
            const bool ended = hipEventQuery(L.done) == hipSuccess;
            const int nf = (int)L.wave.size();
            const int n = L.wave[0].code->n;
            const size_t off_f = lpdec::lp_align((size_t)nf * n);
            const size_t off_o = off_f + lpdec::lp_align(4 * (size_t)nf);
            const size_t off_d = off_o + lpdec::lp_align(8 * (size_t)nf);
            const volatile int32_t *dn = (const volatile int32_t *)(L.out.h + off_d);
            const auto now = std::chrono::steady_clock::now();
            for (int k = 0; k < nf; ++k) {
                if (L.retired[k] || !(dn[k] || ended)) continue;
                std::atomic_thread_fence(std::memory_order_acquire);
                Result r;
                if (dn[k]) {
                    const uint8_t *xh = (const uint8_t *)L.out.h + (size_t)k * n;
                    r.xhat.assign(xh, xh + n);
                    r.flag = ((const volatile int32_t *)(L.out.h + off_f))[k];
                    r.obj = ((const volatile double *)(L.out.h + off_o))[k];
                } else {
                    // the kernel ended without marking this frame
                    r.xhat.assign(n, 0);
                    r.flag = LPDEC_FLAG_NONFINITE;
                }
                r.latency = std::chrono::duration<double>(now - L.wave[k].t_submit).count();
                done.emplace_back(L.wave[k].ticket, std::move(r));
                L.retired[k] = 1;
                ++L.nretired;
            }
            if (!ended) continue;
            // the lane gives its device memory back with the wave's budget: stream-ordered
            // frees on its own stream, which other lanes' kernels do not wait for
            lane_release(L);
            freed_bytes += L.footprint;
            freed_slots += nf;
            L.wave.clear();
            L.busy = false;
        }
        // admission: take a wave for every idle lane while the queue head fits
        struct Launch { Lane *L; size_t need; };
        std::vector<Launch> launches;
        bool any_busy = false, stop = false;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto &d : done) {
                s->results[d.first] = std::move(d.second);
                s->pending.erase(d.first);
            }
            s->in_use -= freed_bytes;
            s->slots_in_use -= freed_slots;
            for (auto &L : s->lanes) {
                if (L.busy || s->queue.empty()) continue;
                // the head request and every later queued request of the same code, in
                // arrival order, while the budget and the slots allow; the others keep their
                // places
                const lpdec_code *code = s->queue.front().code;
                const size_t fp = frame_footprint(code, pt64);
                int nf = 0;
                size_t need = 0;
                for (auto it = s->queue.begin(); it != s->queue.end();) {
                    if (it->code != code) { ++it; continue; }
                    if (s->slots_in_use + nf + 1 > s->max_slots) break;
                    if (s->in_use + need + fp > s->budget) break;
                    need += fp;
                    ++nf;
                    L.wave.push_back(std::move(*it));
                    it = s->queue.erase(it);
                }
                if (nf == 0) break;
                s->in_use += need;
                s->slots_in_use += nf;
                L.busy = true;
                launches.push_back({&L, need});
            }
            stop = s->stop;
        }
        if (!done.empty()) s->cv_done.notify_all();
        for (auto &ln : launches) {
            Lane &L = *ln.L;
            const lpdec_code *code = L.wave[0].code;
            const int nf = (int)L.wave.size();
            const int n = code->n;
            const size_t off_f = lpdec::lp_align((size_t)nf * n);
            const size_t off_o = off_f + lpdec::lp_align(4 * (size_t)nf);
            const size_t off_d = off_o + lpdec::lp_align(8 * (size_t)nf);
            const size_t out_bytes = off_d + 4 * (size_t)nf;
            std::vector<double> g((size_t)nf * n);
            for (int k = 0; k < nf; ++k) std::copy(L.wave[k].gamma.begin(), L.wave[k].gamma.end(), g.begin() + (size_t)k * n);
            // device memory exactly as admitted: the kernel workspace is the wave's footprint
            // (a region the launch cannot grow) and the inputs their own bytes, both allocated on
            // the lane's stream and released when the wave retires
            hipError_t e = lane_alloc(L.ws, ln.need, L.stream);
            if (e == hipSuccess) e = lane_alloc(L.io, 8 * g.size(), L.stream);
            if (e == hipSuccess) e = hostout_ensure(L.out, out_bytes);
            if (e == hipSuccess) {
                // the lane is idle, so nothing reads the previous wave's flags any more
                std::memset(L.out.h + off_d, 0, 4 * (size_t)nf);
                std::atomic_thread_fence(std::memory_order_release);
                e = hipMemcpyAsync(L.io.ptr, g.data(), 8 * g.size(), hipMemcpyHostToDevice, L.stream);
            }
            L.retired.assign(nf, 0);
            L.nretired = 0;
            L.footprint = ln.need;
            lpdec_status st = LPDEC_EDEVICE;
            if (e == hipSuccess) {
                // the copy is ordered before the kernel on the same stream; synchronise it so
                // g can go
                e = hipStreamSynchronize(L.stream);
                st = e == hipSuccess
                         ? decode_batch_impl(s->ctx, code, nf, L.io.ptr, 1, (uint8_t *)L.out.d,
                                             (int32_t *)(L.out.d + off_f), (double *)(L.out.d + off_o),
                                             nullptr, nullptr, nullptr, 0, pt64, L.ws, L.stream,
                                             (int32_t *)(L.out.d + off_d))
                         : LPDEC_EDEVICE;
            }
            if (st == LPDEC_OK) e = hipEventRecord(L.done, L.stream);
            if (st != LPDEC_OK || e != hipSuccess) {
                // report the failure on every frame of the wave and give its budget back
                std::lock_guard<std::mutex> lk(s->mu);
                for (auto &r : L.wave) {
                    Result res;
                    res.xhat.assign(n, 0);
                    res.flag = LPDEC_FLAG_NONFINITE;
                    s->results[r.ticket] = std::move(res);
                    s->pending.erase(r.ticket);
                }
                s->in_use -= L.footprint;
                s->slots_in_use -= nf;
                L.wave.clear();
                L.busy = false;
                lane_release(L);
                s->err = "wave launch failed";
                s->cv_done.notify_all();
            }
        }
        for (auto &L : s->lanes) any_busy |= L.busy;
        if (any_busy) {
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            continue;
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && s->queue.empty()) break;
        if (stop && s->queue.empty()) break;
        s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        if (s->stop && s->queue.empty()) break;
    }
}

// ------------------------------------------------------------------ persistent engines
// Server mode 1. Each code gets an Engine once a request for it arrives; the engine's kernel
// stays resident while requests keep coming and leaves after about 5 ms in which none was
// decoded or waiting (or when the engine is freed), and the server thread launches it again when tickets wait and it has left.
// The thread alone touches the engines and, in this mode, the budget counter in_use.

constexpr int kIdlePolls = 100;   // about 5 ms

hipError_t engine_init(Engine &E, const lpdec_code *code, int W, int R)
{
    using lpdec::lp_align;
    E.code = code;
    E.W = W;
    E.R = R;
    const size_t n = (size_t)code->n;
    E.off_x = lp_align(8 * (size_t)R * n);
    E.off_f = E.off_x + lp_align((size_t)R * n);
    E.off_o = E.off_f + lp_align(4 * (size_t)R);
    E.off_d = E.off_o + lp_align(8 * (size_t)R);
    E.off_c = E.off_d + lp_align(4 * (size_t)R);
    E.slot.resize(R);
    E.used.assign(R, 0);
    hipError_t e = hipStreamCreateWithFlags(&E.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&E.ended, hipEventDisableTiming);
    if (e == hipSuccess) e = hostout_ensure(E.ring, E.off_c + 256);
    if (e == hipSuccess) std::memset(E.ring.h, 0, E.ring.bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&E.claim, 256);
    if (e == hipSuccess) e = hipMemset(E.claim, 0, 256);
    return e;
}

// Asks a resident kernel to leave, waits for it, and frees everything the engine holds.
void engine_free(Engine &E)
{
    if (E.ring.h) __atomic_store_n(E.ctl() + 1, 1, __ATOMIC_RELEASE);
    if (E.stream) (void)hipStreamSynchronize(E.stream);
    ws_free(E.ws);
    if (E.claim) (void)hipFree(E.claim);
    if (E.ring.h) (void)hipHostFree(E.ring.h);
    if (E.ended) (void)hipEventDestroy(E.ended);
    if (E.stream) (void)hipStreamDestroy(E.stream);
    E.claim = nullptr;
    E.ring = HostOut{};
    E.ended = nullptr;
    E.stream = nullptr;
}

lpdec_status engine_launch(lpdec_server *s, Engine &E, int pt64)
{
    Args a{};
    a.mode = lpdec::MODE_SERVE;
    a.gamma = E.ring.d;
    a.gamma_f64 = 1;
    a.xhat = (uint8_t *)(E.ring.d + E.off_x);
    a.flag = (int32_t *)(E.ring.d + E.off_f);
    a.obj = (double *)(E.ring.d + E.off_o);
    a.done = (int32_t *)(E.ring.d + E.off_d);
    a.claim = E.claim;
    a.published = (const int32_t *)(E.ring.d + E.off_c);
    a.stop = (const int32_t *)(E.ring.d + E.off_c) + 1;
    a.share = (const int32_t *)(E.ring.d + E.off_c) + 2;
    // workgroups beyond the current share would leave at once
    a.nframes = std::max(1, std::min(E.W, E.ctl()[2]));
    a.ring = E.R;
    a.idle_polls = kIdlePolls;
    // the previous launch on this stream has ended: it left no ticket held and closed itself
    // (or stopped); clear its busy count and closing flag
    if (hipMemsetAsync(E.claim + 1, 0, 8, E.stream) != hipSuccess) return LPDEC_EDEVICE;
    lpdec_status st = launch(s->ctx, E.code, a, pt64, E.ws, E.stream);
    if (st == LPDEC_OK && hipEventRecord(E.ended, E.stream) != hipSuccess) st = LPDEC_EDEVICE;
    if (st == LPDEC_OK) E.running = true;
    return st;
}

// The engine of a code, created if the budget allows (engines without work are freed first
// when it does not); null if the request has to wait. hip_failed reports an engine that could
// not be set up.
Engine *engine_for(lpdec_server *s, const lpdec_code *code, int pt64, bool &hip_failed)
{
    hip_failed = false;
    for (auto &E : s->engines)
        if (E->code == code) return E.get();
    const size_t fp = frame_footprint(code, pt64);
    const int want = std::min(s->max_slots, s->ncu);
    auto room = [&] { return (long long)((s->budget - s->in_use) / fp); };
    if (room() < want) {
        for (size_t k = 0; k < s->engines.size();) {
            Engine &E = *s->engines[k];
            if (E.outstanding || !E.backlog.empty()) { ++k; continue; }
            engine_free(E);
            s->in_use -= E.footprint;
            s->engines.erase(s->engines.begin() + (long)k);
        }
    }
    const int W = (int)std::min<long long>(want, room());
    if (W < 1) return nullptr;
    auto E = std::make_unique<Engine>();
    const int R = std::max(64, std::min(4096, 2 * s->max_slots));
    if (engine_init(*E, code, W, R) != hipSuccess) {
        engine_free(*E);
        hip_failed = true;
        return nullptr;
    }
    E->footprint = (size_t)W * fp;
    s->in_use += E->footprint;
    s->engines.push_back(std::move(E));
    return s->engines.back().get();
}

void server_loop_persistent(lpdec_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    const int pt64 = precision_for(s->ctx, 1);
    auto failed = [](const Request &r) {
        Result res;
        res.xhat.assign(r.code->n, 0);
        res.flag = LPDEC_FLAG_NONFINITE;
        return std::make_pair(r.ticket, std::move(res));
    };
    std::vector<std::pair<uint64_t, Result>> done;
    while (true) {
        // retire the frames whose done flags are set; an engine whose kernel has ended is
        // marked idle before its flags are read, so that a ticket still without a flag then was
        // published after the workgroups left and waits for the next launch
        int freed = 0;
        const auto now = std::chrono::steady_clock::now();
        for (auto &Ep : s->engines) {
            Engine &E = *Ep;
            if (E.running && hipEventQuery(E.ended) != hipErrorNotReady) E.running = false;
            if (!E.outstanding) continue;
            const int n = E.code->n;
            const volatile int32_t *dn = (const volatile int32_t *)(E.ring.h + E.off_d);
            for (int k = 0; k < E.R; ++k) {
                if (!E.used[k] || !dn[k]) continue;
                std::atomic_thread_fence(std::memory_order_acquire);
                Result r;
                const uint8_t *xh = (const uint8_t *)E.ring.h + E.off_x + (size_t)k * n;
                r.xhat.assign(xh, xh + n);
                r.flag = ((const volatile int32_t *)(E.ring.h + E.off_f))[k];
                r.obj = ((const volatile double *)(E.ring.h + E.off_o))[k];
                r.latency = std::chrono::duration<double>(now - E.slot[k].t_submit).count();
                done.emplace_back(E.slot[k].ticket, std::move(r));
                E.slot[k] = Request{};
                E.used[k] = 0;
                --E.outstanding;
                ++freed;
            }
        }
        // admission: queued requests in arrival order while slots are left
        std::vector<Request> incoming;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto &d : done) {
                s->results[d.first] = std::move(d.second);
                s->pending.erase(d.first);
            }
            s->slots_in_use -= freed;
            while (!s->queue.empty() && s->slots_in_use < s->max_slots) {
                incoming.push_back(std::move(s->queue.front()));
                s->queue.pop_front();
                ++s->slots_in_use;
            }
        }
        if (!done.empty()) s->cv_done.notify_all();
        done.clear();
        size_t k = 0;
        for (; k < incoming.size(); ++k) {
            bool hip_failed = false;
            Engine *E = engine_for(s, incoming[k].code, pt64, hip_failed);
            if (hip_failed) {
                done.push_back(failed(incoming[k]));
                continue;
            }
            if (!E) break;
            E->backlog.push_back(std::move(incoming[k]));
        }
        if (k < incoming.size() || !done.empty()) {
            // requests that wait for budget go back to the head of the queue in their order
            std::lock_guard<std::mutex> lk(s->mu);
            for (size_t j = incoming.size(); j-- > k;) s->queue.push_front(std::move(incoming[j]));
            s->slots_in_use -= (int)(incoming.size() - k);
            for (auto &d : done) {
                s->results[d.first] = std::move(d.second);
                s->pending.erase(d.first);
            }
            s->slots_in_use -= (int)done.size();
            if (!done.empty()) s->err = "engine setup failed";
        }
        if (!done.empty()) s->cv_done.notify_all();
        done.clear();
        // publish into free slots
        bool busy = false;
        int active = 0;
        for (auto &Ep : s->engines) {
            Engine &E = *Ep;
            if (!E.running && !E.outstanding && E.published > (1 << 30) &&
                hipMemset(E.claim, 0, 256) == hipSuccess) {
                // restart the ticket counters long before they could overflow (the device
                // counter first; if that fails both keep counting)
                E.published = 0;
                __atomic_store_n(E.ctl(), 0, __ATOMIC_RELEASE);
            }
            const size_t n = (size_t)E.code->n;
            bool pub = false;
            while (!E.backlog.empty()) {
                const int k = E.published % E.R;
                if (E.used[k]) break;
                Request &r = E.backlog.front();
                std::memcpy(E.ring.h + 8 * (size_t)k * n, r.gamma.data(), 8 * n);
                ((volatile int32_t *)(E.ring.h + E.off_d))[k] = 0;
                E.slot[k] = std::move(r);
                E.backlog.pop_front();
                E.used[k] = 1;
                ++E.outstanding;
                ++E.published;
                pub = true;
            }
            if (pub) __atomic_store_n(E.ctl(), E.published, __ATOMIC_RELEASE);
            active += E.outstanding > 0 || !E.backlog.empty();
        }
        // the compute units are shared evenly among the engines with work (one workgroup per
        // compute unit each); an engine without work keeps its workgroups only while no other
        // has any. Then launch an engine whose kernel has left while tickets wait.
        for (auto &Ep : s->engines) {
            Engine &E = *Ep;
            const bool work = E.outstanding > 0 || !E.backlog.empty();
            const int share = work ? std::max(1, s->ncu / std::max(1, active)) : (active ? 0 : s->ncu);
            if (E.ctl()[2] != share) __atomic_store_n(E.ctl() + 2, share, __ATOMIC_RELAXED);
            if (!E.running && E.outstanding > 0 && engine_launch(s, E, pt64) != LPDEC_OK) {
                for (int j = 0; j < E.R; ++j) {
                    if (!E.used[j]) continue;
                    done.push_back(failed(E.slot[j]));
                    E.slot[j] = Request{};
                    E.used[j] = 0;
                }
                E.outstanding = 0;
                // the device never saw these tickets: count them as claimed
                (void)hipMemcpy(E.claim, &E.published, 4, hipMemcpyHostToDevice);
            }
            busy |= E.outstanding > 0 || !E.backlog.empty();
        }
        if (!done.empty()) {
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto &d : done) {
                s->results[d.first] = std::move(d.second);
                s->pending.erase(d.first);
            }
            s->slots_in_use -= (int)done.size();
            s->err = "engine launch failed";
            s->cv_done.notify_all();
            done.clear();
        }
        if (busy) {
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            continue;
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && s->queue.empty()) break;
        s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        if (s->stop && s->queue.empty()) break;
    }
}

}  // namespace

extern "C" lpdec_status lpdec_server_create(lpdec_ctx *ctx, size_t hbm_budget_bytes, int32_t max_slots,
                                            lpdec_server **out)
{
    if (!ctx || !out) return LPDEC_EINVAL;
    if (max_slots <= 0 || hbm_budget_bytes == 0) return fail(ctx, LPDEC_EINVAL, "budget and max_slots must be > 0");
    (void)hipSetDevice(ctx->device);
    auto *s = new (std::nothrow) lpdec_server();
    if (!s) return LPDEC_ENOMEM;
    s->ctx = ctx;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->mode = ctx->server_mode;
    if (s->mode == 1) {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || ncu < 1)
            ncu = 1;
        s->ncu = ncu;
        s->worker = std::thread(server_loop_persistent, s);
        *out = s;
        return LPDEC_OK;
    }
    s->lanes.resize(ctx->server_streams);
    for (auto &L : s->lanes) {
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
            lpdec_server_destroy(s);
            return fail(ctx, LPDEC_EDEVICE, "stream creation failed");
        }
    }
    s->worker = std::thread(server_loop, s);
    *out = s;
    return LPDEC_OK;
}

extern "C" lpdec_status lpdec_server_submit(lpdec_server *s, const lpdec_code *code, const double *gamma,
                                            uint64_t *ticket)
{
    if (!s || !code || !gamma || !ticket || code->ctx != s->ctx) return LPDEC_EINVAL;
    Request r;
    r.code = code;
    r.gamma.assign(gamma, gamma + code->n);
    r.t_submit = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return LPDEC_EINVAL;
        if (frame_footprint(code, precision_for(s->ctx, 1)) > s->budget) return LPDEC_ENOMEM;
        r.ticket = s->next_ticket++;
        *ticket = r.ticket;
        s->pending[r.ticket] = 1;
        s->queue.push_back(std::move(r));
    }
    s->cv_work.notify_one();
    return LPDEC_OK;
}

extern "C" lpdec_status lpdec_server_poll(lpdec_server *s, uint64_t ticket, uint8_t *xhat, int32_t *flag,
                                          double *objective, double *latency_s)
{
    if (!s) return LPDEC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return s->pending.count(ticket) ? LPDEC_EBUSY : LPDEC_ENOTFOUND;
    if (xhat) std::memcpy(xhat, it->second.xhat.data(), it->second.xhat.size());
    if (flag) *flag = it->second.flag;
    if (objective) *objective = it->second.obj;
    if (latency_s) *latency_s = it->second.latency;
    s->results.erase(it);
    return LPDEC_OK;
}

extern "C" lpdec_status lpdec_server_drain(lpdec_server *s)
{
    if (!s) return LPDEC_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->pending.empty(); });
    return LPDEC_OK;
}

extern "C" lpdec_status lpdec_server_destroy(lpdec_server *s)
{
    if (!s) return LPDEC_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto &E : s->engines) engine_free(*E);
    for (auto &L : s->lanes) {
        if (L.stream) {
            lane_release(L);
            (void)hipStreamSynchronize(L.stream);
        }
        if (L.out.h) (void)hipHostFree(L.out.h);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    delete s;
    return LPDEC_OK;
}
