// Device side of the decoder: one workgroup owns one frame and runs every step of the
// hot path on it -- cut search (Algorithm 2), cut management (Algorithm 3 / MALP-B), the
// primal-dual interior-point iteration (Sec. IV-B), the triangular-set search (Algorithm 7)
// with its level schedule, and PCG (Algorithm 4) with the preconditioner of Sec. V.
//
// Index spaces of one frame:
//   checks j in [0, m): a check "has a cut" when vmask[j] != 0 (V of its single parity
//     inequality, Theorem 3); LP rows are the checks with a cut, in ascending order;
//     every row vector is stored in check space (length m) and is 0 off the LP rows.
//   columns c in [0, n+m): standard column i < n (the flipped variable x_i), slack column
//     n+j of the row of check j (present only when check j has a cut).
//   A entry of (row j, standard column i at position k of row j):
//     sg[i] * (+1 if bit k of vmask[j] is set, else -1); the slack entry is +1.
//
// Everything a PCG iteration or a step of Algorithm 7 reads sits in LDS: per LP the row and
// column lists of A with the signs folded in (rlist, clist), per interior-point iteration the
// instruction lists of the two triangular solves in level order (bins, fins). Global memory
// holds the FP64 interior-point state, touched a few times per interior-point iteration.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lpdec_common.hpp"

namespace lpdec {

#define LPD_INLINE __device__ __forceinline__

constexpr int kMaxWaves = 4;    // up to 256 threads per frame
constexpr uint16_t kEnd = 0xFFFF;

// -------------------------------------------------------------------- list entries
// bit 15: the coefficient is -1; bit 14: the entry refers to a row value; bits 0..13: index.
LPD_INLINE uint16_t enc(int idx, bool neg, bool rowref = false)
{
    return (uint16_t)((neg ? 0x8000u : 0u) | (rowref ? 0x4000u : 0u) | (unsigned)idx);
}
LPD_INLINE int e_idx(uint16_t e) { return e & 0x3FFF; }
LPD_INLINE bool e_neg(uint16_t e) { return (e & 0x8000u) != 0; }
LPD_INLINE bool e_row(uint16_t e) { return (e & 0x4000u) != 0; }
template <typename T>
LPD_INLINE T sgnv(uint16_t e, T v) { return e_neg(e) ? -v : v; }

// Triangular-solve slot entries: (index << 1) | negative. In the PCG the index addresses
// one vector space, s (rows, [0, m)) followed by t (columns, m + c) and one slot that is
// always 0 (m + n + m), which also pads every slot; the header entry of a slot holds the
// row and the sign of its diagonal coefficient.
LPD_INLINE uint16_t ben(int idx, bool neg) { return (uint16_t)((idx << 1) | (neg ? 1 : 0)); }
LPD_INLINE int b_idx(uint16_t e) { return e >> 1; }
LPD_INLINE bool b_neg(uint16_t e) { return (e & 1u) != 0; }
LPD_INLINE double flip(double v, bool neg)
{
    return __hiloint2double(__double2hiint(v) ^ (neg ? (int)0x80000000 : 0), __double2loint(v));
}
LPD_INLINE float flip(float v, bool neg) { return __uint_as_float(__float_as_uint(v) ^ (neg ? 0x80000000u : 0u)); }
// v with sign neg, or +0 when keep is false (integer masks, no branch)
LPD_INLINE double maskflip(double v, bool neg, bool keep)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned long long sg = (unsigned long long)neg << 63;
    return __longlong_as_double((long long)((b ^ sg) & (0ull - (unsigned long long)keep)));
}
LPD_INLINE float maskflip(float v, bool neg, bool keep)
{
    const uint32_t b = __float_as_uint(v), sg = (uint32_t)neg << 31;
    return __uint_as_float((b ^ sg) & (0u - (uint32_t)keep));
}

// Sum over aligned groups of G lanes (4, 8 or 16) with DPP: quad_perm [1,0,3,2] and
// [2,3,0,1] within quads, then row_half_mirror and row_mirror. Every lane of a group ends
// with the same sum (each step adds two operands in either order). All lanes must be active.
// (every row and bank is enabled and every source lane exists, so no old value is needed)
template <int CTRL>
LPD_INLINE double dpp_mov(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// The value of a double in one lane (a wave-uniform lane index), for every lane.
LPD_INLINE double lp_readlane_d(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Accumulator of the FP64 16x16x4 matrix-core product
typedef double lp_d4 __attribute__((ext_vector_type(4)));
template <int CTRL>
LPD_INLINE float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
// Makes the compiler materialise v here, so that a load feeding v stays where it is issued
// (beside the other loads of a step) instead of being sunk into the branch that uses it.
LPD_INLINE void pin(double v) { asm volatile("" ::"v"(v)); }
LPD_INLINE void pin(float v) { asm volatile("" ::"v"(v)); }

template <int G, typename T>
LPD_INLINE T gsum(T v)
{
    v = v + dpp_mov<0xB1>(v);
    v = v + dpp_mov<0x4E>(v);
    if constexpr (G >= 8) v = v + dpp_mov<0x141>(v);
    if constexpr (G >= 16) v = v + dpp_mov<0x140>(v);
    return v;
}

// A chunk of list entries read with one load: 8 entries (16 bytes) of a row-type slot or 4
// entries (8 bytes) of a column-type slot. Every entry of a chunk is processed without a
// data-dependent exit, so the gathers it feeds are issued together.
struct Ch8 {
    uint32_t w[4];
    static constexpr int K = 8;
};
struct Ch4 {
    uint32_t w[2];
    static constexpr int K = 4;
};
LPD_INLINE void ldch(Ch8 &c, const uint16_t *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    c.w[0] = v.x; c.w[1] = v.y; c.w[2] = v.z; c.w[3] = v.w;
}
LPD_INLINE void ldch(Ch4 &c, const uint16_t *p)
{
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    c.w[0] = v.x; c.w[1] = v.y;
}
template <typename CH>
LPD_INLINE void endch(CH &c)
{
#pragma unroll
    for (int k = 0; k < CH::K / 2; ++k) c.w[k] = 0xFFFFFFFFu;
}
template <typename CH>
LPD_INLINE uint16_t at(const CH &c, int k) { return (uint16_t)(c.w[k >> 1] >> ((k & 1) << 4)); }

// v with the sign of entry e applied, or +0 when keep is false, computed with integer masks:
// with no branch for the compiler to sink the load of v into, the loads of consecutive entries
// are issued back to back and overlap their latencies.
LPD_INLINE double sgn_keep(double v, uint16_t e, bool keep)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned long long sg = (unsigned long long)(e & 0x8000u) << 48;
    const unsigned long long km = 0ull - (unsigned long long)keep;
    return __longlong_as_double((long long)((b ^ sg) & km));
}
LPD_INLINE float sgn_keep(float v, uint16_t e, bool keep)
{
    const uint32_t b = __float_as_uint(v);
    const uint32_t sg = (uint32_t)(e & 0x8000u) << 16;
    const uint32_t km = 0u - (uint32_t)keep;
    return __uint_as_float((b ^ sg) & km);
}

// Signed value of one list entry (0 for the end marker); the load is unconditional (index 0
// for the marker).
template <typename T, typename V>
LPD_INLINE T sgather(uint16_t e, const V *base)
{
    const bool ok = e != kEnd;
    return sgn_keep((T)base[ok ? e_idx(e) : 0], e, ok);
}

// -------------------------------------------------------------------- wave reductions
// Inclusive scan inside rows of 16 lanes (row_shr 1, 2, 4, 8), then across rows
// (row_bcast 15 into rows 1 and 3, row_bcast 31 into rows 2 and 3); lane 63 ends up with the
// reduction of the wave, which readlane hands to every lane. All 64 lanes must be active.
template <int CTRL, int ROWM>
LPD_INLINE uint32_t dpp(uint32_t identity, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, ROWM, 0xF, false);
}

#define LPD_DPP_SCAN(OP, ID, V)           \
    V = OP(V, dpp<0x111, 0xF>(ID, V));    \
    V = OP(V, dpp<0x112, 0xF>(ID, V));    \
    V = OP(V, dpp<0x114, 0xF>(ID, V));    \
    V = OP(V, dpp<0x118, 0xF>(ID, V));    \
    V = OP(V, dpp<0x142, 0xA>(ID, V));    \
    V = OP(V, dpp<0x143, 0xC>(ID, V));

LPD_INLINE uint32_t op_max_u(uint32_t a, uint32_t b) { return a > b ? a : b; }
LPD_INLINE uint32_t op_add_u(uint32_t a, uint32_t b) { return a + b; }
LPD_INLINE uint32_t op_add_f(uint32_t a, uint32_t b) { return __float_as_uint(__uint_as_float(a) + __uint_as_float(b)); }

LPD_INLINE uint32_t wave_max_u32(uint32_t v)
{
    LPD_DPP_SCAN(op_max_u, 0u, v)
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// max over lanes 0..15 (row 0) for every lane: row_shr scan, then lane 15
LPD_INLINE uint32_t row16_max_u32(uint32_t v)
{
    v = op_max_u(v, dpp<0x111, 0xF>(0u, v));
    v = op_max_u(v, dpp<0x112, 0xF>(0u, v));
    v = op_max_u(v, dpp<0x114, 0xF>(0u, v));
    v = op_max_u(v, dpp<0x118, 0xF>(0u, v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
}

// max of 64-bit keys: high words first, then the low words of the lanes holding that high word
LPD_INLINE unsigned long long wave_max_u64(unsigned long long k)
{
    const uint32_t hi = wave_max_u32((uint32_t)(k >> 32));
    const uint32_t lo = wave_max_u32((uint32_t)(k >> 32) == hi ? (uint32_t)k : 0u);
    return ((unsigned long long)hi << 32) | lo;
}

LPD_INLINE float wave_sum(float v)
{
    uint32_t q = __float_as_uint(v);
    LPD_DPP_SCAN(op_add_f, 0u, q)
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)q, 63));
}

LPD_INLINE int wave_sum(int v)
{
    uint32_t q = (uint32_t)v;
    LPD_DPP_SCAN(op_add_u, 0u, q)
    return __builtin_amdgcn_readlane((int)q, 63);
}

LPD_INLINE double wave_sum(double v)
{
#define LPD_DSTEP(CTRL, ROWM)                                                   \
    {                                                                         \
        const uint32_t lo = dpp<CTRL, ROWM>(0u, (uint32_t)__double2loint(v)); \
        const uint32_t hi = dpp<CTRL, ROWM>(0u, (uint32_t)__double2hiint(v)); \
        v = v + __hiloint2double((int)hi, (int)lo);                           \
    }
    LPD_DSTEP(0x111, 0xF)
    LPD_DSTEP(0x112, 0xF)
    LPD_DSTEP(0x114, 0xF)
    LPD_DSTEP(0x118, 0xF)
    LPD_DSTEP(0x142, 0xA)
    LPD_DSTEP(0x143, 0xC)
#undef LPD_DSTEP
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

template <typename T>
LPD_INLINE T wave_max_t(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

template <typename T>
LPD_INLINE T wave_min_t(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

// -------------------------------------------------------------------- block reductions
// Shared scratch for reductions: kMaxWaves slots per value, up to 4 values.
struct Scratch {
    double d[4 * kMaxWaves];
    unsigned long long u64[2];
    int i[8];
};

// Block-wide sums of K values. The leading barrier also ends the caller's previous phase.
template <int K, typename T>
LPD_INLINE void block_sum(T (&v)[K], Scratch *s)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (nw == 1) return;
    T *buf = reinterpret_cast<T *>(s->d);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) buf[k * kMaxWaves + wv] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        T a = 0;
        for (int w = 0; w < nw; ++w) a += buf[k * kMaxWaves + w];
        v[k] = a;
    }
    __syncthreads();
}

template <typename T>
LPD_INLINE T block_sum1(T v, Scratch *s)
{
    T a[1] = {v};
    block_sum<1>(a, s);
    return a[0];
}

// [0] summed, [1] maximised (values >= 0) over the block.
template <typename T>
LPD_INLINE void block_summax(T (&v)[2], Scratch *s)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v[0] = wave_sum(v[0]);
    v[1] = wave_max_t(v[1]);
    __syncthreads();
    if (nw == 1) return;
    T *buf = reinterpret_cast<T *>(s->d);
    if (lane == 0) { buf[wv] = v[0]; buf[kMaxWaves + wv] = v[1]; }
    __syncthreads();
    T a = 0, b = 0;
    for (int w = 0; w < nw; ++w) {
        a += buf[w];
        b = buf[kMaxWaves + w] > b ? buf[kMaxWaves + w] : b;
    }
    v[0] = a;
    v[1] = b;
    __syncthreads();
}

LPD_INLINE double block_max_d(double v, Scratch *s)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_max_t(v);
    __syncthreads();
    if (nw == 1) return v;
    if (lane == 0) s->d[wv] = v;
    __syncthreads();
    double a = s->d[0];
    for (int w = 1; w < nw; ++w) a = s->d[w] > a ? s->d[w] : a;
    __syncthreads();
    return a;
}

LPD_INLINE void block_min2(double &a, double &b, Scratch *s)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    a = wave_min_t(a);
    b = wave_min_t(b);
    __syncthreads();
    if (nw == 1) return;
    if (lane == 0) { s->d[wv] = a; s->d[kMaxWaves + wv] = b; }
    __syncthreads();
    a = s->d[0];
    b = s->d[kMaxWaves];
    for (int w = 1; w < nw; ++w) {
        a = s->d[w] < a ? s->d[w] : a;
        b = s->d[kMaxWaves + w] < b ? s->d[kMaxWaves + w] : b;
    }
    __syncthreads();
}

LPD_INLINE int block_or(int v, Scratch *s)
{
    const unsigned long long bal = __ballot(v != 0);
    const int nw = blockDim.x >> 6;
    __syncthreads();
    if (nw == 1) return bal != 0ull;
    if (threadIdx.x == 0) s->i[0] = 0;
    __syncthreads();
    if ((threadIdx.x & 63) == 0 && bal) atomicOr(&s->i[0], 1);
    __syncthreads();
    const int r = s->i[0];
    __syncthreads();
    return r;
}

LPD_INLINE int block_max_i(int v, Scratch *s)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_max_t(v);
    __syncthreads();
    if (nw == 1) return v;
    if (lane == 0) reinterpret_cast<int *>(s->d)[wv] = v;
    __syncthreads();
    int a = reinterpret_cast<int *>(s->d)[0];
    for (int w = 1; w < nw; ++w) {
        const int b = reinterpret_cast<int *>(s->d)[w];
        a = b > a ? b : a;
    }
    __syncthreads();
    return a;
}

// Exclusive scan over cnt[0..len) in place (wave 0 does it, chunks of 64); the others wait.
LPD_INLINE void block_exscan(int *cnt, int len)
{
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int carry = 0;
        for (int base = 0; base < len; base += 64) {
            const int v = (base + lane < len) ? cnt[base + lane] : 0;
            int incl = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(incl, o, 64);
                if (lane >= o) incl += t;
            }
            if (base + lane < len) cnt[base + lane] = carry + incl - v;
            carry += __shfl(incl, 63, 64);
        }
        if (lane == 0) cnt[len] = carry;
    }
    __syncthreads();
}

// Ordering key of Algorithm 7: float weight descending, then column index ascending,
// packed so that a larger 64-bit integer means "preferred"; 0 means "no column".
LPD_INLINE unsigned long long mts_key(float w, int c)
{
    return ((unsigned long long)__float_as_uint(w) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)c);
}
LPD_INLINE int mts_key_col(unsigned long long k) { return (int)(0xFFFFFFFFu - (unsigned)(k & 0xFFFFFFFFull)); }

// -------------------------------------------------------------------- one frame
template <typename PT>
struct Frame {
    CodeView cd;
    Opts o;
    int m, n, RW, CW, tid, nt;
    Scratch *sc;
    // hot
    PT *h, *r, *v, *l, *s, *idm, *om, *t, *d2f;
    uint16_t *rlist, *clist, *bins, *fins;
    int16_t *pair, *pairrow, *lbv, *lfv, *order;
    int *boff, *foff;
    uint8_t *deg;
    int8_t *sg;
    uint32_t *vmask;
    uint8_t *rank;       // rank of a column among the columns of its lane (Algorithm 7)
    uint16_t *lcol;      // the columns of each lane by rank: lcol[r * 64 + lane]
    uint32_t *lmask;     // available columns of each lane by rank: word w at lmask[w * 64 + lane]
    uint8_t *rdeg;       // Algorithm 8: remaining columns of each row
    uint32_t *r1m;       // Algorithm 8: rows with one remaining column, one bit per check
    int RWC, CWC, MW;    // chunks per row slot, per column slot; mask words per lane
    // cold
    double *x, *z, *dx, *dz, *rc, *tq, *d2, *y, *dy, *rb, *w, *b, *rho, *f64, *u, *g;
    double *c64[8];   // FP64 PCG vectors for escalated solves, and a copy of dy
    double *st64;     // s | t | 0 of the escalated FP64 PCG
    int *ridx;        // dense fallback: LP row index of each check
    double *colk, *qd;   // dense fallback: work vector, the p x p matrix (null when absent)
    double *ldsd;        // dense fallback: factor of the diagonal tile, reciprocals, vector block (LDS)
    uint8_t *active;
    uint32_t *vprev;     // cut of each check in the previous LP of this decode
    uint32_t *vback;     // cut of each check in the LP before the previous one
    bool have_prev;      // an LP of this decode has been solved
    // level counts of the current preconditioner, LP rows
    int nlb, nlf, p;
    int Z;                 // index of the zero slot of the PCG vector space (n + 2m)
    long long ticks_pcg;   // clock ticks spent inside pcg() during the current decode

    LPD_INLINE void bind(const Args &a, const CodeView &cv, char *hot, char *cold, Scratch *scr)
    {
        cd = cv; o = a.o; m = cd.m; n = cd.n; RW = a.plan.rw; CW = a.plan.cw;
        RWC = RW / 8; CWC = CW / 4; MW = a.plan.maskwords;
        tid = threadIdx.x; nt = blockDim.x; sc = scr;
        ticks_pcg = 0;
        const Plan &P = a.plan;
        h = (PT *)(hot + P.h); r = (PT *)(hot + P.r); v = (PT *)(hot + P.v); l = (PT *)(hot + P.l);
        s = (PT *)(hot + P.st); idm = (PT *)(hot + P.idm); om = (PT *)(hot + P.om);
        t = s + m; d2f = (PT *)(hot + P.d2f);
        Z = n + 2 * m;
        st64 = (double *)(cold + P.st64);
        ridx = (int *)(cold + P.ridx);
        colk = (double *)(cold + P.colk);
        qd = P.dense_on ? (double *)(cold + P.dense) : nullptr;
        rlist = (uint16_t *)(hot + P.rlist); clist = (uint16_t *)(hot + P.clist);
        bins = (uint16_t *)(hot + P.bins); fins = (uint16_t *)(hot + P.fins);
        pair = (int16_t *)(hot + P.pair); pairrow = (int16_t *)(hot + P.pairrow);
        lbv = (int16_t *)(hot + P.lbv); lfv = (int16_t *)(hot + P.lfv); order = (int16_t *)(hot + P.order);
        boff = (int *)(hot + P.boff); foff = (int *)(hot + P.foff);
        deg = (uint8_t *)(hot + P.deg); sg = (int8_t *)(hot + P.sg); vmask = (uint32_t *)(hot + P.vmask);
        rank = (uint8_t *)(hot + P.rank); lcol = (uint16_t *)(hot + P.lcol); lmask = (uint32_t *)(hot + P.lmask);
        rdeg = (uint8_t *)(hot + P.rdeg); r1m = (uint32_t *)(hot + P.r1);
        x = (double *)(cold + P.x); z = (double *)(cold + P.z); dx = (double *)(cold + P.dx);
        dz = (double *)(cold + P.dz); rc = (double *)(cold + P.rc); tq = (double *)(cold + P.tq);
        d2 = (double *)(cold + P.d2); y = (double *)(cold + P.y); dy = (double *)(cold + P.dy);
        rb = (double *)(cold + P.rb); w = (double *)(cold + P.w); b = (double *)(cold + P.b);
        rho = (double *)(cold + P.rho); f64 = (double *)(cold + P.f64);
        u = (double *)(cold + P.u); g = (double *)(cold + P.g);
        for (int k = 0; k < 8; ++k) c64[k] = (double *)(cold + P.c64 + (size_t)k * lp_align(8 * (size_t)m));
        active = (uint8_t *)(cold + P.active);
        vprev = (uint32_t *)(cold + P.vprev);
        vback = (uint32_t *)(cold + P.vback);
        have_prev = false;
    }

    LPD_INLINE bool cut(int j) const { return vmask[j] != 0u; }
    LPD_INLINE bool colpresent(int c) const { return c < n || vmask[c - n] != 0u; }
    // A entry of row j at position k (variable i), from H, V and the channel signs
    LPD_INLINE int aent(int j, int k, int i) const
    {
        return ((vmask[j] >> k) & 1u) ? (int)sg[i] : -(int)sg[i];
    }
    LPD_INLINE double cost(int c) const { return c < n ? fabs(g[c]) : 0.0; }

    // Row and column lists of the LP's A with the signs folded in (rebuilt for every LP).
    LPD_INLINE void build_lists()
    {
        for (int j = tid; j < m; j += nt) {
            uint16_t *L = rlist + (size_t)j * RW;
            if (cut(j)) {
                const int e0 = cd.rowptr[j], d = cd.rowptr[j + 1] - e0;
                for (int k = 0; k < RW; ++k) {
                    if (k < d) {
                        const int i = cd.col[e0 + k];
                        L[k] = enc(i, aent(j, k, i) < 0);
                    } else {
                        L[k] = kEnd;
                    }
                }
            } else {
                for (int k = 0; k < RW; ++k) L[k] = kEnd;
            }
        }
        for (int i = tid; i < n; i += nt) {
            uint16_t *L = clist + (size_t)i * CW;
            int c = 0;
            for (int e = cd.colptr[i]; e < cd.colptr[i + 1]; ++e) {
                const int vv = cd.vlist[e], j = vv >> 5;
                if (cut(j)) L[c++] = enc(j, aent(j, vv & 31, i) < 0);
            }
            for (; c < CW; ++c) L[c] = kEnd;
        }
        __syncthreads();
    }

    // (A x)_j over the columns of row j, slack included (row j has a cut)
    template <typename T, typename V>
    LPD_INLINE T row_dot(int j, const V *xq) const
    {
        T acc = (T)xq[n + j];
        for (int ch = 0; ch < RWC; ++ch) {
            Ch8 E;
            ldch(E, rlist + (size_t)j * RW + 8 * ch);
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += sgather<T>(at(E, k), xq);
        }
        return acc;
    }
    // (A^T y)_i for standard column i, y in check space
    template <typename T, typename V>
    LPD_INLINE T col_dot(int i, const V *yy) const
    {
        T acc = 0;
        for (int ch = 0; ch < CWC; ++ch) {
            Ch4 E;
            ldch(E, clist + (size_t)i * CW + 4 * ch);
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += sgather<T>(at(E, k), yy);
        }
        return acc;
    }

    // ------------------------------------------------------------ Algorithm 2
    // Violated parity inequality of check j at u (FP64). Returns 1 when violated.
    LPD_INLINE int find_cut(int j, uint32_t &V, double &lhs) const
    {
        const int e0 = cd.rowptr[j], d = cd.rowptr[j + 1] - e0;
        uint32_t S = 0;
        int cnt = 0, ks = 0;
        double best = 0.0;
        for (int k = 0; k < d; ++k) {
            const double uk = u[cd.col[e0 + k]];
            if (uk > 0.5) { S |= 1u << k; ++cnt; }
            const double a = fabs(uk - 0.5);
            if (k == 0 || a < best) { best = a; ks = k; }
        }
        V = (cnt & 1) ? S : (S ^ (1u << ks));
        double acc = 0.0;
        for (int k = 0; k < d; ++k) {
            const double uk = u[cd.col[e0 + k]];
            acc += ((V >> k) & 1u) ? (1.0 - uk) : uk;
        }
        lhs = acc;
        return acc < 1.0 - o.tau_viol;
    }

    // ------------------------------------------------------------ Algorithm 7 + levels
    LPD_INLINE float wt(const float *wk, int c) const { return wk ? wk[c] : (float)d2f[c]; }
    LPD_INLINE bool present(int c) const { return c < n || cut(c - n); }
    LPD_INLINE unsigned long long colkey(const float *wk, int c) const { return mts_key(wt(wk, c), c); }
    LPD_INLINE void mask_set(int c, bool on)
    {
        const int r = rank[c];
        uint32_t *wp = &lmask[(r >> 5) * 64 + (c & 63)];
        if (on) atomicOr(wp, 1u << (r & 31));
        else atomicAnd(wp, ~(1u << (r & 31)));
    }

    // Column-wise greedy search for the triangular set (Algorithm 7), exactly as stated:
    // p times, take the degree-1 column with the largest key (weight, then lowest index)
    // and eliminate the only row it still has.
    //   Lane l of wave 0 owns the columns c = l + 64 r. Before the search the columns of each
    // lane are ranked by key (lcol lists them by rank) and a bit mask per lane marks the
    // available ones (degree 1, not taken; a slack column while its row is live). A lane's
    // best column is its lowest set bit, the chosen column the wave maximum of the lanes'
    // keys. Eliminating a row clears the bits of the chosen column and of the row's slack,
    // and the row's other columns lose one degree: 2 -> 1 sets their bit, 1 -> 0 clears it.
    // Fills pair (column of each row), pairrow (row of each chosen standard column), order
    // (rows in elimination order), lfv (forward-substitution level) and lbv
    // (back-substitution level). Returns p.
    //   With k0 > 0 the search only completes a set: the rows matched so far (order[0..k0),
    //   their pair, pairrow and lbv) stay, the search runs over the unmatched rows and the
    //   columns none of whose rows is matched (the matrix A-bar of the triangular expansion
    //   in Sec. V-B), and its rows follow in order from position k0.
    LPD_INLINE int mts(const float *wk, int k0 = 0)
    {
        for (int i = tid; i < n; i += nt) {
            int dg = 0;
            bool excl = false;
            for (int ch = 0; ch < CWC; ++ch) {
                Ch4 E;
                ldch(E, clist + (size_t)i * CW + 4 * ch);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint16_t e = at(E, k);
                    dg += e != kEnd;
                    excl |= k0 > 0 && e != kEnd && pair[e_idx(e)] >= 0;
                }
            }
            deg[i] = (uint8_t)(excl ? 0 : dg);
            if (!k0) pairrow[i] = -1;
        }
        int pl = 0;
        for (int j = tid; j < m; j += nt) {
            if (!k0) { pair[j] = -1; lbv[j] = -1; }
            if (pair[j] < 0) { lfv[j] = -1; lbv[j] = -1; }
            pl += cut(j) && pair[j] < 0;
        }
        for (int k = tid; k < 64 * MW; k += nt) lmask[k] = 0u;
        pl = block_sum1(pl, sc);
        if (!k0) p = pl;
        // rank of each present column among the present columns of its lane
        for (int c = tid; c < n + m; c += nt) {
            if (!present(c)) continue;
            const unsigned long long kc = colkey(wk, c);
            int r = 0;
            for (int c2 = c & 63; c2 < n + m; c2 += 64) {
                const unsigned long long k2 = present(c2) ? colkey(wk, c2) : 0ull;
                r += k2 > kc;
            }
            rank[c] = (uint8_t)r;
            lcol[r * 64 + (c & 63)] = (uint16_t)c;
        }
        __syncthreads();
        for (int c = tid; c < n + m; c += nt)
            if (present(c) && (c >= n ? pair[c - n] < 0 : deg[c] == 1)) mask_set(c, true);
        __syncthreads();
        int done = 0;   // rows eliminated (wave 0)
        if (tid < 64) {
            const int lane = tid;
            const int le = lane < RW ? lane : RW - 1;   // entry of the eliminated row this lane reads
            for (int step = 0; step < pl; ++step) {
                __builtin_amdgcn_wave_barrier();
                int r = -1;
                for (int wd = 0; wd < MW && r < 0; ++wd) {
                    const uint32_t bits = lmask[wd * 64 + lane];
                    if (bits) r = wd * 32 + __builtin_ctz(bits);
                }
                const int cl = r >= 0 ? (int)lcol[r * 64 + lane] : 0;
                const unsigned long long kl = colkey(wk, cl);
                const unsigned long long mine = r >= 0 ? kl : 0ull;
                const unsigned long long K = wave_max_u64(mine);
                if (K == 0ull) break;   // no degree-1 column: cannot happen while rows remain
                const int c = mts_key_col(K);
                // the row of c: its only live row; the other rows give the forward level.
                // Lane k < CW reads entry k of the column's list (CW <= 16)
                int row = c - n, L = 0;
                if (c < n) {
                    const uint16_t ce = lane < CW ? clist[(size_t)c * CW + lane] : kEnd;
                    const bool okc = ce != kEnd;
                    const int jc = okc ? e_idx(ce) : 0;
                    const int pjc = pair[jc], ljc = lfv[jc];
                    const unsigned long long live = __ballot(okc && pjc < 0);
                    if (!live) break;   // a degree-1 column always has its live row
                    row = __builtin_amdgcn_readlane(jc, __ffsll((long long)live) - 1);
                    L = (int)row16_max_u32(okc && pjc >= 0 ? (uint32_t)(ljc + 1) : 0u);
                }
                // everything the updates read, loaded together
                const uint16_t e = rlist[(size_t)row * RW + le];
                const bool ok = lane < RW && e != kEnd;
                const int i = ok ? e_idx(e) : 0;
                const int pri = pairrow[i], dgi = deg[i] - 1, rki = rank[i];
                const int rkc = rank[c], rks = rank[n + row];
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) {
                    pair[row] = (int16_t)c;
                    lfv[row] = (int16_t)L;
                    order[k0 + step] = (int16_t)row;
                    if (c < n) pairrow[c] = (int16_t)row;
                    atomicAnd(&lmask[(rkc >> 5) * 64 + (c & 63)], ~(1u << (rkc & 31)));
                    if (c != n + row) atomicAnd(&lmask[(rks >> 5) * 64 + ((n + row) & 63)], ~(1u << (rks & 31)));
                }
                // eliminate the row: its waiting columns lose one degree
                if (ok && i != c && pri < 0 && dgi >= 0) {
                    deg[i] = (uint8_t)dgi;
                    uint32_t *wp = &lmask[(rki >> 5) * 64 + (i & 63)];
                    if (dgi == 1) atomicOr(wp, 1u << (rki & 31));
                    else if (dgi == 0) atomicAnd(wp, ~(1u << (rki & 31)));
                }
                done = step + 1;
            }
        }
        __syncthreads();
        // back-substitution levels: a row depends on the rows of the other chosen columns in
        // it, all eliminated later. The dependencies are listed in parallel (into bins, which
        // the level build rewrites afterwards), then wave 0 walks the rows in reverse
        // elimination order with the next row's list prefetched.
        uint16_t *dep = bins;
        for (int j = tid; j < m; j += nt) {
            if (!cut(j)) continue;
            const int c = pair[j];
            for (int k = 0; k < RW; ++k) {
                const uint16_t e = rlist[(size_t)j * RW + k];
                const int i = e != kEnd ? e_idx(e) : 0;
                const int pr = pairrow[i];
                dep[(size_t)j * RW + k] = (e != kEnd && i != c && pr >= 0) ? (uint16_t)pr : kEnd;
            }
        }
        __syncthreads();
        if (tid < 64 && done > 0) {
            const int lane = tid;
            const int le = lane < RW ? lane : RW - 1;
            int rown = order[k0 + done - 1];
            uint16_t dn = dep[(size_t)rown * RW + le];
            for (int step = done - 1; step >= 0; --step) {
                const int row = rown;
                const uint16_t dd = lane < RW ? dn : kEnd;
                if (step > 0) {
                    rown = order[k0 + step - 1];
                    dn = dep[(size_t)rown * RW + le];
                }
                const int lv = lbv[dd != kEnd ? dd : 0];
                const int L = (int)wave_max_u32(dd != kEnd ? (uint32_t)(lv + 1) : 0u);
                if (lane == 0) lbv[row] = (int16_t)L;
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        return pl;
    }

    // Row-wise greedy search for the triangular set (Algorithm 8) with diagonal expansion.
    //   The residual matrix holds the LP rows and the columns that still have entries there.
    //   rdeg counts each row's remaining columns, r1m marks the rows with exactly one, and the
    //   per-lane masks of Algorithm 7 mark the remaining columns, ranked per lane by
    //   (weight, index) ascending so that a lane's lowest set bit is its lightest column.
    //   Wave 0 runs the steps: the lowest-indexed row of degree 1 is matched with its only
    //   remaining column (the row's lanes find it); without such a row the lightest remaining
    //   column (wave minimum) is removed unmatched. Removing a column lowers the degree of
    //   each of its rows. Rows left unmatched then take their slack, in ascending order.
    //   A_M is lower triangular in matching order, so back-substitution dependencies point to
    //   rows matched earlier and forward ones to rows matched later: the levels are computed
    //   walking the order forward and backward respectively. Fills pair, pairrow, order, lbv,
    //   lfv as mts() does. Returns p.
    LPD_INLINE unsigned long long rowkey(const float *wk, int c) const
    {
        return ((unsigned long long)__float_as_uint(wt(wk, c)) << 32) | (unsigned long long)(unsigned)c;
    }
    LPD_INLINE bool col_left(int c) const
    {
        const int r = rank[c];
        return (lmask[(r >> 5) * 64 + (c & 63)] >> (r & 31)) & 1u;
    }
    //   With expand = 1 (triangular expansion) the unmatched rows are matched instead by the
    //   column-wise search over the columns none of whose rows is matched (mts() with k0 =
    //   the rows matched so far): A_M = [A_M1 0; B A_M2]. Back-substitution levels are then
    //   walked forward over the row-wise rows and backward over the others (inside mts()),
    //   forward-substitution levels the other way round.
    LPD_INLINE int mts_row(const float *wk, int expand = 0)
    {
        const int r1w = (m + 31) >> 5;
        for (int i = tid; i < n; i += nt) {
            int dg = 0;
            for (int ch = 0; ch < CWC; ++ch) {
                Ch4 E;
                ldch(E, clist + (size_t)i * CW + 4 * ch);
#pragma unroll
                for (int k = 0; k < 4; ++k) dg += at(E, k) != kEnd;
            }
            deg[i] = (uint8_t)dg;
            pairrow[i] = -1;
        }
        int pl = 0;
        for (int j = tid; j < m; j += nt) {
            pair[j] = -1; lfv[j] = -1; lbv[j] = -1;
            int d = 0;
            if (cut(j)) {
                ++pl;
                d = 1;   // the slack
                for (int k = 0; k < RW; ++k) d += rlist[(size_t)j * RW + k] != kEnd;
            }
            rdeg[j] = (uint8_t)d;
        }
        for (int k = tid; k < 64 * MW; k += nt) lmask[k] = 0u;
        for (int k = tid; k < r1w; k += nt) r1m[k] = 0u;
        pl = block_sum1(pl, sc);
        p = pl;
        // rank of each remaining column among the remaining columns of its lane, ascending key
        for (int c = tid; c < n + m; c += nt) {
            if (!present(c) || (c < n && deg[c] == 0)) continue;
            const unsigned long long kc = rowkey(wk, c);
            int r = 0;
            for (int c2 = c & 63; c2 < n + m; c2 += 64)
                r += present(c2) && (c2 >= n || deg[c2] > 0) && rowkey(wk, c2) < kc;
            rank[c] = (uint8_t)r;
            lcol[r * 64 + (c & 63)] = (uint16_t)c;
        }
        __syncthreads();
        for (int c = tid; c < n + m; c += nt)
            if (present(c) && (c >= n || deg[c] > 0)) mask_set(c, true);
        __syncthreads();
        if (tid < 64) {
            const int lane = tid;
            int k = 0, live = pl;   // rows with remaining columns
            while (live > 0) {
                __builtin_amdgcn_wave_barrier();
                int cand = 0x7FFFFFFF;
                for (int wd = lane; wd < r1w; wd += 64) {
                    const uint32_t b = r1m[wd];
                    if (b) { cand = wd * 32 + __builtin_ctz(b); break; }
                }
                const int jr = wave_min_t(cand);
                int c;
                if (jr != 0x7FFFFFFF) {
                    // the only remaining column of row jr: lane q < RW looks at entry q, lane
                    // RW at the slack
                    int cl = -1;
                    if (lane < RW) {
                        const uint16_t e = rlist[(size_t)jr * RW + lane];
                        cl = e != kEnd ? e_idx(e) : -1;
                    } else if (lane == RW) {
                        cl = n + jr;
                    }
                    c = wave_max_t(cl >= 0 && col_left(cl) ? cl : -1);
                    if (c < 0) break;   // cannot happen: a degree-1 row has its column
                    if (lane == 0) {
                        pair[jr] = (int16_t)c;
                        order[k] = (int16_t)jr;
                        if (c < n) pairrow[c] = (int16_t)jr;
                    }
                    ++k;
                } else {
                    int r = -1;
                    for (int wd = 0; wd < MW && r < 0; ++wd) {
                        const uint32_t bits = lmask[wd * 64 + lane];
                        if (bits) r = wd * 32 + __builtin_ctz(bits);
                    }
                    const unsigned long long key = r >= 0 ? rowkey(wk, (int)lcol[r * 64 + lane]) : ~0ull;
                    const unsigned long long K = ~wave_max_u64(~key);
                    if (K == ~0ull) break;   // no column left: cannot happen while rows have some
                    c = (int)(unsigned)(K & 0xFFFFFFFFull);
                }
                // remove column c: its rows lose one degree
                const int rk = rank[c];
                int jj = -1;
                if (c >= n) {
                    jj = lane == 0 ? c - n : -1;
                } else if (lane < CW) {
                    const uint16_t e = clist[(size_t)c * CW + lane];
                    jj = e != kEnd ? e_idx(e) : -1;
                }
                const int nd = jj >= 0 ? (int)rdeg[jj] - 1 : -1;
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) atomicAnd(&lmask[(rk >> 5) * 64 + (c & 63)], ~(1u << (rk & 31)));
                if (jj >= 0) {
                    rdeg[jj] = (uint8_t)nd;
                    uint32_t *wp = &r1m[jj >> 5];
                    if (nd == 1) atomicOr(wp, 1u << (jj & 31));
                    else if (nd == 0) atomicAnd(wp, ~(1u << (jj & 31)));
                }
                live -= __popcll(__ballot(nd == 0));
            }
            // diagonal expansion: the unmatched rows with a cut take their slack, ascending
            __builtin_amdgcn_wave_barrier();
            for (int base = 0; base < m && !expand; base += 64) {
                const int j = base + lane;
                const bool un = j < m && cut(j) && pair[j] < 0;
                const unsigned long long bal = __ballot(un);
                if (un) {
                    pair[j] = (int16_t)(n + j);
                    order[k + __popcll(bal & ((1ull << lane) - 1ull))] = (int16_t)j;
                }
                k += __popcll(bal);
            }
            // levels: back-substitution dependencies (the rows of the row's other matched
            // columns) were matched earlier, forward ones (the other rows of the row's column)
            // later
            __builtin_amdgcn_wave_barrier();
            mts_row_back_levels(k);
            if (!expand) mts_row_fwd_levels(k);
            if (lane == 0) sc->i[1] = k;
        }
        __syncthreads();
        if (expand) {
            const int k1 = sc->i[1];
            __syncthreads();
            mts(wk, k1);
            if (tid < 64) mts_row_fwd_levels(k1);
            __syncthreads();
        }
        return pl;
    }

    // Back-substitution levels of the first k rows of order when A_M is lower triangular in
    // that order: walking forward, a row's dependencies (the rows of its other matched columns)
    // are already set. Wave 0.
    LPD_INLINE void mts_row_back_levels(int k)
    {
        const int lane = tid & 63;
        for (int step = 0; step < k; ++step) {
            const int row = order[step];
            int L = 0;
            if (lane < RW) {
                const uint16_t e = rlist[(size_t)row * RW + lane];
                const int i = e != kEnd ? e_idx(e) : -1;
                const int pr = i >= 0 && i != pair[row] ? (int)pairrow[i] : -1;
                L = pr >= 0 ? lbv[pr] + 1 : 0;
            }
            L = (int)row16_max_u32((uint32_t)L);
            if (lane == 0) lbv[row] = (int16_t)L;
            __builtin_amdgcn_wave_barrier();
        }
    }

    // Forward-substitution levels of the first k rows of order, walking backward (their
    // dependencies, the other rows of the matched column, come later or are already set).
    // Wave 0.
    LPD_INLINE void mts_row_fwd_levels(int k)
    {
        const int lane = tid & 63;
        for (int step = k - 1; step >= 0; --step) {
            const int row = order[step], c = pair[row];
            int L = 0;
            if (c < n && lane < CW) {
                const uint16_t e = clist[(size_t)c * CW + lane];
                const int jj = e != kEnd ? e_idx(e) : -1;
                L = jj >= 0 && jj != row ? lfv[jj] + 1 : 0;
            }
            L = (int)row16_max_u32((uint32_t)L);
            if (lane == 0) lfv[row] = (int16_t)L;
            __builtin_amdgcn_wave_barrier();
        }
    }

    // ------------------------------------------------------------ Algorithm 6 + Algorithm 5
    // Column states of the incremental search, kept in rank[]: in M, candidate of the current
    // test, matched by the current peeling.
    static constexpr uint8_t kInM = 1, kCand = 2, kGone = 4;

    // Triangulation Step (Algorithm 5) on S = the columns marked kInM or kCand: peeling in
    // rounds. Each row with exactly one remaining column of S at the start of a round proposes
    // that column; a column proposed by several rows goes to the lowest-indexed one, and every
    // row of a matched column loses one degree. Rows matched in one round depend only on
    // columns matched in earlier rounds, so any order within a round keeps A_S lower
    // triangular. Fills pair, pairrow (standard columns) and order. Returns the number of
    // columns matched: |S| when the set passes.
    LPD_INLINE int peel_set()
    {
        int *rd = boff;            // remaining columns of S in each row
        int *owner = (int *)s;     // lowest row proposing each column in the current round
        int16_t *prop = lbv;       // column each row proposes in the current round
        for (int c = tid; c < n + m; c += nt) {
            rank[c] &= (uint8_t)(kInM | kCand);
            owner[c] = 0x7FFFFFFF;
            if (c < n) pairrow[c] = -1;
        }
        __syncthreads();
        for (int j = tid; j < m; j += nt) {
            pair[j] = -1;
            int d = 0;
            if (cut(j)) {
                d = rank[n + j] != 0;
                for (int k = 0; k < RW; ++k) {
                    const uint16_t e = rlist[(size_t)j * RW + k];
                    d += e != kEnd && rank[e_idx(e)] != 0;
                }
            }
            rd[j] = d;
        }
        if (tid == 0) sc->i[3] = 0;
        __syncthreads();
        int matched = 0;
        for (;;) {
            for (int j = tid; j < m; j += nt) {
                int c = -1;
                if (pair[j] < 0 && rd[j] == 1) {
                    if (rank[n + j] == kInM || rank[n + j] == kCand) c = n + j;
                    for (int k = 0; k < RW; ++k) {
                        const uint16_t e = rlist[(size_t)j * RW + k];
                        const int i = e != kEnd ? e_idx(e) : 0;
                        if (e != kEnd && (rank[i] == kInM || rank[i] == kCand)) c = i;
                    }
                    if (c >= 0) atomicMin(&owner[c], j);
                }
                prop[j] = (int16_t)c;
            }
            __syncthreads();
            for (int j = tid; j < m; j += nt) {
                const int c = prop[j];
                if (c < 0 || owner[c] != j) continue;
                pair[j] = (int16_t)c;
                order[atomicAdd(&sc->i[3], 1)] = (int16_t)j;
                rank[c] |= kGone;
                if (c >= n) {
                    atomicSub(&rd[c - n], 1);
                } else {
                    pairrow[c] = (int16_t)j;
                    for (int k = 0; k < CW; ++k) {
                        const uint16_t e = clist[(size_t)c * CW + k];
                        if (e != kEnd) atomicSub(&rd[e_idx(e)], 1);
                    }
                }
            }
            __syncthreads();
            const int tot = sc->i[3];
            if (tot == matched) break;
            matched = tot;
        }
        __syncthreads();
        return matched;
    }

    // Marks srt[pos + t], t < kk, as candidates for t < cand and with state `rest` otherwise.
    LPD_INLINE void inc_mark(const uint16_t *srt, int pos, int kk, int cand, uint8_t rest)
    {
        __syncthreads();
        for (int t = tid; t < kk; t += nt) rank[srt[pos + t]] = t < cand ? kCand : rest;
        __syncthreads();
    }

    // Incremental greedy search for the triangular set (Algorithm 6): the LP's columns in key
    // order (weight descending, index ascending), each added to M while M with it passes the
    // Triangulation Step, until M has p columns. Equivalent batched form (Sec. V-C adds
    // several columns per call): a block of the next kk columns is tested at once; if M with
    // the whole block passes, so does M with every prefix of it, and all are added; otherwise
    // bisection finds the shortest failing prefix, whose columns before the last are added and
    // whose last column is dropped, exactly as one-at-a-time testing would. The block doubles
    // after a pass and halves after a failure. Fills pair, pairrow, order, lbv, lfv; A_M is
    // lower triangular in matching order. Returns p; calls counts Triangulation Steps.
    LPD_INLINE int mts_inc(const float *wk, int &calls)
    {
        uint16_t *srt = lcol;
        int pl = 0, ql = 0;
        for (int j = tid; j < m; j += nt) pl += cut(j);
        for (int c = tid; c < n + m; c += nt) {
            rank[c] = 0;
            if (c < n) pairrow[c] = -1;
            if (!present(c)) continue;
            ++ql;
            const unsigned long long kc = colkey(wk, c);
            int r = 0;
            for (int c2 = 0; c2 < n + m; ++c2) r += present(c2) && colkey(wk, c2) > kc;
            srt[r] = (uint16_t)c;
        }
        for (int j = tid; j < m; j += nt) { pair[j] = -1; lbv[j] = -1; lfv[j] = -1; }
        pl = block_sum1(pl, sc);
        ql = block_sum1(ql, sc);
        p = pl;
        int msz = 0, pos = 0, blk = 16;
        calls = 0;
        while (msz < pl && pos < ql) {
            const int kk = min(min(blk, ql - pos), pl - msz);
            inc_mark(srt, pos, kk, kk, 0);
            ++calls;
            if (peel_set() == msz + kk) {
                inc_mark(srt, pos, kk, 0, kInM);
                msz += kk;
                pos += kk;
                blk *= 2;
                continue;
            }
            int lo = 0, hi = kk;   // M with the first lo passes, with the first hi fails
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                inc_mark(srt, pos, kk, mid, 0);
                ++calls;
                if (peel_set() == msz + mid) lo = mid;
                else hi = mid;
            }
            // the first lo columns join M, column lo is dropped, the rest wait for later tests
            inc_mark(srt, pos, kk, 0, 0);
            if (lo > 0) inc_mark(srt, pos, lo, 0, kInM);
            msz += lo;
            pos += lo + 1;
            blk = max(1, kk >> 1);
        }
        // the pairing of the final set, then the levels of the lower-triangular solves
        peel_set();
        if (tid < 64) {
            mts_row_back_levels(msz);
            mts_row_fwd_levels(msz);
        }
        __syncthreads();
        return pl;
    }

    // The preconditioning set of the context's PRECOND from the weights d2f: Algorithm 7 (1),
    // Algorithm 8 with diagonal (2) or triangular (3) expansion, Algorithm 6 (5), else the
    // slack columns.
    LPD_INLINE int find_precond_set()
    {
        int calls = 0;
        if (o.precond == 1) mts(nullptr);
        else if (o.precond == 2 || o.precond == 3) mts_row(nullptr, o.precond - 2);
        else if (o.precond == 5) mts_inc(nullptr, calls);
        else slack_basis();
        return calls;
    }

    // The slack columns as preconditioning set (A_M = I): used when Algorithm 7 is off.
    LPD_INLINE void slack_basis()
    {
        for (int i = tid; i < n; i += nt) pairrow[i] = -1;
        int pl = 0;
        for (int j = tid; j < m; j += nt) {
            const bool cj = cut(j);
            pair[j] = cj ? (int16_t)(n + j) : (int16_t)-1;
            lbv[j] = cj ? 0 : -1;
            lfv[j] = cj ? 0 : -1;
            pl += cj;
        }
        p = block_sum1(pl, sc);
    }

    // Rows grouped by level, each with its instruction list. Back-substitution level L holds
    // slots [L ? boff[L-1] : 0, boff[L]) of bins (RW entries per slot), forward level L
    // slots [L ? foff[L-1] : 0, foff[L]) of fins (CW entries per slot), entries encoded by
    // ben(). Slot header: the row and the sign of its diagonal entry. Back entries: the other
    // M-columns of the row as references to their rows (index < m, coefficient negated), the
    // columns outside M (the slack included) as column references (index m + column).
    // Forward entries: the other rows of the paired column (coefficient negated).
    LPD_INLINE void build_levels()
    {
        int mb = -1, mf = -1;
        for (int j = tid; j < m; j += nt) { mb = max(mb, (int)lbv[j]); mf = max(mf, (int)lfv[j]); }
        mb = block_max_i(mb, sc);
        mf = block_max_i(mf, sc);
        nlb = mb + 1;
        nlf = mf + 1;
        for (int k = tid; k <= m; k += nt) { boff[k] = 0; foff[k] = 0; }
        __syncthreads();
        for (int j = tid; j < m; j += nt) {
            if (lbv[j] >= 0) atomicAdd(&boff[lbv[j]], 1);
            if (lfv[j] >= 0) atomicAdd(&foff[lfv[j]], 1);
        }
        block_exscan(boff, nlb);
        block_exscan(foff, nlf);
        for (int j = tid; j < m; j += nt) {
            if (lbv[j] < 0) continue;
            const int c = pair[j];
            // back-substitution slot
            {
                uint16_t *B = bins + (size_t)atomicAdd(&boff[lbv[j]], 1) * RW;
                const uint16_t *L = rlist + (size_t)j * RW;
                bool dneg = false;
                int q = 1;
                for (int k = 0; k < RW; ++k) {
                    const uint16_t e = L[k];
                    if (e == kEnd) break;
                    const int i = e_idx(e);
                    if (i == c) { dneg = e_neg(e); continue; }
                    if (pairrow[i] >= 0) B[q++] = ben(pairrow[i], !e_neg(e));
                    else B[q++] = ben(m + i, e_neg(e));
                }
                if (c != n + j) B[q++] = ben(m + n + j, false);
                for (; q < RW; ++q) B[q] = ben(Z, false);
                B[0] = ben(j, dneg);
            }
            // forward-substitution slot
            {
                uint16_t *F = fins + (size_t)atomicAdd(&foff[lfv[j]], 1) * CW;
                bool dneg = false;
                int q = 1;
                if (c < n) {
                    const uint16_t *L = clist + (size_t)c * CW;
                    for (int k = 0; k < CW; ++k) {
                        const uint16_t e = L[k];
                        if (e == kEnd) break;
                        const int jj = e_idx(e);
                        if (jj == j) { dneg = e_neg(e); continue; }
                        F[q++] = ben(jj, !e_neg(e));
                    }
                }
                for (; q < CW; ++q) F[q] = ben(Z, false);
                F[0] = ben(j, dneg);
            }
        }
        __syncthreads();
        // boff[L] / foff[L] now end level L; mark the levels that fit one pass of wave 0
        if (tid < 64) {
            mark_small(boff, nlb, 64 / RW);
            mark_small(foff, nlf, 64 / CW);
        }
        __syncthreads();
    }

    // Wave 0: sets kSmallLevel on the level ends off[0..nlev) of levels with at most `fit` slots.
    LPD_INLINE void mark_small(int *off, int nlev, int fit)
    {
        const int lane = tid & 63;
        for (int base = 0; base < nlev; base += 64) {
            const int L = base + lane;
            bool small = false;
            int e = 0;
            if (L < nlev) {
                e = off[L] & kOffMask;
                const int s0 = L ? (off[L - 1] & kOffMask) : 0;
                small = e - s0 <= fit;
            }
            __builtin_amdgcn_wave_barrier();
            if (L < nlev && small) off[L] = e | kSmallLevel;
            __builtin_amdgcn_wave_barrier();
        }
    }

    // ------------------------------------------------------------ triangular solves
    // The preconditioning set M pairs every LP row j with one column pair[j]; A_M (rows by
    // paired columns) is triangular after permutation with entries +-1 (Sec. V). Vectors over
    // M's columns are stored at the row each column is paired with.
    //
    // Level-by-level sweep over the slots of one triangular solve, one lane per slot entry:
    // groups of G lanes (G = slot width) take the slots of a level. Every lane computes the
    // value of its entry (gather; the header lane q = 0 contributes 0) and whatever the row's
    // finish needs (pre), the group sums the values with DPP, and the header lane finishes
    // the row. Levels are separated by a barrier; level bounds are read two levels ahead and
    // each lane's entry of the next level one level ahead.
    //   A level with at most 64 / G slots fits one pass of wave 0. A run of such levels (most
    // levels of the long dependency chains of late interior-point iterations hold a few rows)
    // is swept by wave 0 alone: its LDS accesses are processed in program order, so a level
    // needs only the wait for the previous level's stores, not a workgroup barrier; the other
    // waves meet wave 0 at the end of the run. build_levels() marks such levels in off[].
    static constexpr int kSmallLevel = 1 << 30;
    static constexpr int kOffMask = kSmallLevel - 1;

    //   A step gathers the value of its lane's entry from vec (with MASKED an index of m or
    // above contributes 0; the header lane and lanes past the level gather a zero) and the
    // header lane loads the row's own operands (pre, from the row index; other lanes load row
    // 0's); only after all these loads are issued (a scheduling barrier keeps them together,
    // so one wait covers them) are the signs applied, the operands combined (mid, off the
    // path of the group sum), the group summed and the row finished.
    template <int G, bool MASKED, typename T, typename V, typename PF, typename MF, typename FF>
    LPD_INLINE void gsweep(const uint16_t *slots, const int *off, int nlev, const V *vec, PF pre, MF mid,
                           FF finish)
    {
        if (nlev <= 0) return;
        const int g = tid / G, q = tid - g * G, ng = nt / G;
        const uint16_t zero = ben(Z, false);
        auto step = [&](bool valid, uint16_t e) {
            const int bi = b_idx(e);
            const bool ok = valid && q != 0 && (!MASKED || bi < m);
            const bool head = valid && q == 0;
            // the row's operands first, the gather last: waiting for the gather then covers
            // every load of the step
            const auto pc = pre(head ? bi : 0);
            T v = (T)vec[ok ? bi : (MASKED ? 0 : Z)];
            __builtin_amdgcn_sched_barrier(0);
            // unmasked, a lane without an entry has gathered the zero element: only the sign
            // is applied
            v = MASKED ? maskflip(v, b_neg(e), ok) : flip(v, b_neg(e));
            const auto pm = mid(pc);   // the row's operands combined, beside the group sum
            const T sum = gsum<G>(v);
            finish(head, e, pm, sum);
        };
        int L = 0, kA = 0, raw = off[0];
        uint16_t cur = !(raw & kSmallLevel) && g < (raw & kOffMask) ? slots[g * G + q] : zero;
        while (L < nlev) {
            if (raw & kSmallLevel) {
                if (tid < 64) {
                    // level l: slots [a, b) with entry e; the end of level l + 1 (raw1) is known
                    // one level ahead and its first entry is loaded during level l, so that
                    // the only dependent LDS access on the chain is the gather of a level
                    // (bounds are the same in every lane: readfirstlane keeps them in scalar
                    // registers, so the loop control is scalar)
                    //   Every load of the loop is unconditional (a lane past its level reads
                    // the level's first slot and its step is invalid; a bound past the last
                    // level reads the last one and is not used), so the loop has no branches
                    // around loads.
                    const int nl = __builtin_amdgcn_readfirstlane(nlev);
                    int l = __builtin_amdgcn_readfirstlane(L), a = __builtin_amdgcn_readfirstlane(kA);
                    int b = __builtin_amdgcn_readfirstlane(raw & kOffMask);
                    uint16_t e = slots[(a + g < b ? a + g : a) * G + q];
                    int raw1 = __builtin_amdgcn_readfirstlane(off[l + 1 < nl ? l + 1 : l]);
                    // nothing in flight on entry: the loop head then needs no wait for the
                    // previous level's store
                    __builtin_amdgcn_s_waitcnt(0xc07f);
                    for (;;) {
                        const bool more = l + 1 < nl && (raw1 & kSmallLevel) != 0;
                        const int nb = raw1 & kOffMask;
                        const uint16_t en = slots[(more && b + g < nb ? b + g : a) * G + q];
                        const int raw2v = off[l + 2 < nl ? l + 2 : nl - 1];
                        step(a + g < b, e);
                        const int raw2 = __builtin_amdgcn_readfirstlane(raw2v);
                        if (!more) break;
                        // the next level's gathers must see the level's stores. In LDS they do
                        // without a wait (the LDS executes one wave's instructions in issue
                        // order); stores to global memory (arenas that do not fit in LDS) are
                        // waited for (vmcnt 0, LDS counter untouched)
                        __builtin_amdgcn_s_waitcnt(0x0f70);
                        __builtin_amdgcn_wave_barrier();
                        ++l;
                        a = b;
                        b = nb;
                        e = en;
                        raw1 = raw2;
                    }
                    if (tid == 0) sc->i[4] = l + 1;
                }
                __syncthreads();
                L = sc->i[4];
                kA = L > 0 ? off[L - 1] & kOffMask : 0;
                raw = L < nlev ? off[L] : 0;
                cur = L < nlev && !(raw & kSmallLevel) && kA + g < (raw & kOffMask) ? slots[(kA + g) * G + q] : zero;
                continue;
            }
            const int kB = raw & kOffMask;
            const int nraw = L + 1 < nlev ? off[L + 1] : 0;
            const uint16_t nxt = L + 1 < nlev && !(nraw & kSmallLevel) && kB + g < (nraw & kOffMask)
                                     ? slots[(kB + g) * G + q] : zero;
            step(kA + g < kB, cur);
            for (int kb = kA + ng; kb < kB; kb += ng) {
                const int k = kb + g;
                step(k < kB, k < kB ? slots[k * G + q] : zero);
            }
            __syncthreads();
            ++L;
            kA = kB;
            raw = nraw;
            cur = nxt;
        }
    }

    // Back-substitution out = A_M^-1 u (levels ascending); out has m entries, only the row
    // references of the slots are used.
    template <int G, typename T, typename UF>
    LPD_INLINE void back_sub_g(T *out, UF u_of_row)
    {
        gsweep<G, true, T>(
            bins, boff, nlb, out,
            [&](int j) { return (T)u_of_row(j); },
            [](T u0) { return u0; },
            [&](bool head, uint16_t e, T u0, T sum) {
                if (head) {
                    const T acc = u0 + sum;
                    out[b_idx(e)] = b_neg(e) ? -acc : acc;
                }
            });
    }
    template <typename T, typename UF>
    LPD_INLINE void back_sub(T *out, UF u_of_row)
    {
        if (RW == 8) back_sub_g<8>(out, u_of_row);
        else back_sub_g<16>(out, u_of_row);
    }

    // Forward substitution out = A_M^-T e (out in row space, m entries; levels ascending).
    template <int G, typename T, typename EF>
    LPD_INLINE void fwd_sub_g(T *out, EF e_of_row)
    {
        gsweep<G, true, T>(
            fins, foff, nlf, out,
            [&](int j) { return (T)e_of_row(j); },
            [](T e0) { return e0; },
            [&](bool head, uint16_t e, T e0, T sum) {
                if (head) {
                    const T acc = e0 + sum;
                    out[b_idx(e)] = b_neg(e) ? -acc : acc;
                }
            });
    }
    template <typename T, typename EF>
    LPD_INLINE void fwd_sub(T *out, EF e_of_row)
    {
        if (CW == 4) fwd_sub_g<4>(out, e_of_row);
        else if (CW == 8) fwd_sub_g<8>(out, e_of_row);
        else fwd_sub_g<16>(out, e_of_row);
    }

    LPD_INLINE bool in_M(int c) const { return c < n ? pairrow[c] >= 0 : pair[c - n] == c; }

    // ------------------------------------------------------------ Algorithm 4
    // PCG on (A D^2 A^T) y = w with M = A_M D_M^2 A_M^T, applied in split form: with
    // L = A_M D_M, CG runs on (I + N N^T) v = L^-1 w, N = L^-1 A_N D_N (A_N, D_N: the columns
    // outside M), and y = L^-T v. In exact arithmetic this produces the iterates of the
    // left-preconditioned Algorithm 4; the large weights of the preconditioning set never
    // multiply a vector, which keeps FP32 arithmetic usable on the ill-conditioned systems
    // of the late interior-point iterations.
    //
    // V holds the vectors of one precision T: r (on entry L^-1 w, then the residual), v (the
    // solution in the transformed space, from 0), h, l, s (work), t (columns), idm (1/d of
    // the column paired with each row), om (sqrt(x z) of that column) and dsq (d^2 of every
    // column).
    // Stops at maxit, when h^T (I + N N^T) h <= 0, and either (xi_stop > 0) when
    // max_j om_j |r_j| <= xi_stop -- the residual L r of the Newton system then perturbs the
    // complementarity equation by Z_M A_M^-1 L r = Z_M D_M r, whose entries are om_j r_j --
    // or (xi_stop = 0) when ||r|| <= tol ||r0||.
    template <typename T>
    struct CG {
        T *r, *v, *h, *l, *s, *t, *idm, *om, *dsq;
    };

    template <typename T>
    LPD_INLINE int pcg(const CG<T> &V, T tol, T xi_stop, int maxit)
    {
        if (RW == 8) {
            if (CW == 4) return pcg_g<T, 8, 4>(V, tol, xi_stop, maxit);
            if (CW == 8) return pcg_g<T, 8, 8>(V, tol, xi_stop, maxit);
            return pcg_g<T, 8, 16>(V, tol, xi_stop, maxit);
        }
        if (CW == 4) return pcg_g<T, 16, 4>(V, tol, xi_stop, maxit);
        if (CW == 8) return pcg_g<T, 16, 8>(V, tol, xi_stop, maxit);
        return pcg_g<T, 16, 16>(V, tol, xi_stop, maxit);
    }

    // V.s and V.t are one vector space (t = s + m) whose element Z is 0; the slot entries
    // index it directly, so the sweeps need no masks.
    template <typename T, int GB, int GF>
    LPD_INLINE int pcg_g(const CG<T> &V, T tol, T xi_stop, int maxit)
    {
        T rr = 0;
        if (tid == 0) V.s[Z] = (T)0;
        for (int j = tid; j < m; j += nt) { V.h[j] = V.r[j]; rr += V.r[j] * V.r[j]; }
        rr = block_sum1(rr, sc);
        if (!(rr > (T)0)) return 0;
        const T stop = tol * tol * rr;
        T *const S = V.s;
        struct HI { T h, i; };   // the row's h and 1/d of its paired column
        int it = 0;
        while (it < maxit) {
            // s = A_M^-T (D_M^-1 h)
            gsweep<GF, false, T>(
                fins, foff, nlf, S,
                [&](int j) { return HI{V.h[j], V.idm[j]}; },
                [](HI hi) { return hi.h * hi.i; },
                [&](bool head, uint16_t e, T e0, T sum) {
#pragma clang fp contract(off)
                    if (head) {
                        const T acc = e0 + sum;
                        S[b_idx(e)] = b_neg(e) ? -acc : acc;
                    }
                });
            // t = D_N^2 A_N^T s on the columns outside M
            for (int c = tid; c < n + m; c += nt) {
                if (c < n) {
                    if (pairrow[c] < 0) V.t[c] = V.dsq[c] * col_dot<T>(c, S);
                } else {
                    const int j = c - n;
                    if (cut(j) && pair[j] != c) V.t[c] = V.dsq[c] * S[j];
                }
            }
            __syncthreads();
            // f = A_M^-1 (A_N t) over s; l = h + D_M^-1 f
            gsweep<GB, false, T>(
                bins, boff, nlb, S,
                [&](int j) { return HI{V.h[j], V.idm[j]}; },
                [](HI hi) { return hi; },
                [&](bool head, uint16_t e, HI hi, T sum) {
                    if (head) {
                        const int j = b_idx(e);
                        const T fj = b_neg(e) ? -sum : sum;
                        S[j] = fj;
                        V.l[j] = hi.h + fj * hi.i;
                    }
                });
            // h^T l in row order: the rows' slots within a level are placed by atomics, so a
            // sum taken in the sweep would depend on that placement
            T hl = 0;
            for (int j = tid; j < m; j += nt)
                if (cut(j)) hl += V.h[j] * V.l[j];
            hl = block_sum1(hl, sc);
            if (!(hl > (T)0)) break;
            const T alpha = rr / hl;
            T a2[2] = {0, 0};   // ||r||^2, max_j om_j |r_j|
            for (int j = tid; j < m; j += nt) {
                if (!cut(j)) continue;
                V.v[j] += alpha * V.h[j];
                const T rj = V.r[j] - alpha * V.l[j];
                V.r[j] = rj;
                a2[0] += rj * rj;
                const T e = V.om[j] * (rj < 0 ? -rj : rj);
                a2[1] = e > a2[1] ? e : a2[1];
            }
            block_summax(a2, sc);
            const T rr2 = a2[0];
            ++it;
            if (xi_stop > (T)0 ? a2[1] <= xi_stop : rr2 <= stop) break;
            const T beta = rr2 / rr;
            rr = rr2;
            for (int j = tid; j < m; j += nt) V.h[j] = V.r[j] + beta * V.h[j];
            __syncthreads();
        }
        return it;
    }

    // PCG iteration cap of one round. PCG_MAXIT > 0 is used as given; 0 (automatic) gives a
    // PCG attempt at least 300 iterations, with which PCG finishes about nine in ten Newton
    // systems of the n=1024 workload (FP64 vectors), and for large LPs about twice the cost of
    // the dense fallback (one dense solve costs about p^2 / 7000 PCG iterations: its work grows
    // as p^3, a PCG iteration's as p); 500 without the fallback. Inside the IPM a round that
    // reaches the cap hands the system to the dense solve.
    LPD_INLINE int pcg_cap() const
    {
        if (o.pcg_maxit > 0) return o.pcg_maxit;
        if (!qd) return 500;
        const double pp = (double)p;
        const double cap = pp * pp / 3500.0;
        return cap < 300.0 ? 300 : (cap > 2000.0 ? 2000 : (int)cap);
    }

    // One refinement round in precision T: r = L^-1 rho, PCG, dy += L^-T v (transforms in
    // FP64). Returns the PCG iterations.
    template <typename T>
    LPD_INLINE int cg_round(const CG<T> &V, double tol, double xi_stop)
    {
        back_sub<double>(f64, [&](int j) { return rho[j]; });
        for (int j = tid; j < m; j += nt) {
            const bool cj = cut(j);
            V.r[j] = cj ? (T)(f64[j] / sqrt(d2[pair[j]])) : (T)0;
            V.v[j] = 0; V.l[j] = 0; V.h[j] = 0; V.s[j] = 0;
            if (cj) {
                V.idm[j] = (T)(1.0 / sqrt(d2[pair[j]]));
                V.om[j] = (T)sqrt(x[pair[j]] * z[pair[j]]);
            }
        }
        __syncthreads();
        const long long t0 = wall_clock64();
        const int its = pcg<T>(V, (T)tol, (T)xi_stop, pcg_cap());
        ticks_pcg += wall_clock64() - t0;
        fwd_sub<double>(f64, [&](int j) { return (double)V.v[j] / sqrt(d2[pair[j]]); });
        for (int j = tid; j < m; j += nt)
            if (cut(j)) dy[j] += f64[j];
        __syncthreads();
        return its;
    }

    // delta = A_M^-1 rho (FP64, at the paired rows, into f64); returns max_j z_j |delta_j|,
    // the largest perturbation of the complementarity equation that rho causes.
    LPD_INLINE double xi_max()
    {
        back_sub<double>(f64, [&](int j) { return rho[j]; });
        double e = 0.0;
        for (int j = tid; j < m; j += nt)
            if (cut(j)) e = fmax(e, z[pair[j]] * fabs(f64[j]));
        return block_max_d(e, sc);
    }

    // rho = w - Q dy in FP64 (Q = A D^2 A^T, D^2 = d2); returns ||rho||^2.
    LPD_INLINE double residual64()
    {
        for (int i = tid; i < n; i += nt) tq[i] = d2[i] * col_dot<double>(i, dy);
        __syncthreads();
        double nr2 = 0.0;
        for (int j = tid; j < m; j += nt) {
            if (!cut(j)) continue;
            double acc = d2[n + j] * dy[j];
            for (int ch = 0; ch < RWC; ++ch) {
                Ch8 E;
                ldch(E, rlist + (size_t)j * RW + 8 * ch);
#pragma unroll
                for (int k = 0; k < 8; ++k) acc += sgather<double>(at(E, k), tq);
            }
            const double rj = w[j] - acc;
            rho[j] = rj;
            nr2 += rj * rj;
        }
        return block_sum1(nr2, sc);
    }

    // Algorithm 4 without a preconditioner (M = I), in FP64, on the current residual rho: the
    // CG baseline of the comparison in Sec. VI-B (PRECOND 4). Stops at ||r|| <= tol ||rho||,
    // at the round's cap or when h^T Q h <= 0; adds the correction to dy. Returns the
    // iterations.
    LPD_INLINE int plain_cg_round(double tol)
    {
        double *const r = c64[0], *const h = c64[1], *const l = c64[2], *const xv = c64[3];
        double rr = 0.0;
        for (int j = tid; j < m; j += nt) {
            const double rj = cut(j) ? rho[j] : 0.0;
            r[j] = rj;
            h[j] = rj;
            xv[j] = 0.0;
            rr += rj * rj;
        }
        rr = block_sum1(rr, sc);
        const double stop = tol * tol * rr;
        const int maxit = pcg_cap();
        int it = 0;
        while (it < maxit && rr > 0.0) {
            // l = A D^2 A^T h
            for (int i = tid; i < n; i += nt) tq[i] = d2[i] * col_dot<double>(i, h);
            __syncthreads();
            double hl = 0.0;
            for (int j = tid; j < m; j += nt) {
                if (!cut(j)) continue;
                double acc = d2[n + j] * h[j];
                for (int ch = 0; ch < RWC; ++ch) {
                    Ch8 E;
                    ldch(E, rlist + (size_t)j * RW + 8 * ch);
#pragma unroll
                    for (int k = 0; k < 8; ++k) acc += sgather<double>(at(E, k), tq);
                }
                l[j] = acc;
                hl += h[j] * acc;
            }
            hl = block_sum1(hl, sc);
            if (!(hl > 0.0)) break;
            const double alpha = rr / hl;
            double rr2 = 0.0;
            for (int j = tid; j < m; j += nt) {
                if (!cut(j)) continue;
                xv[j] += alpha * h[j];
                const double rj = r[j] - alpha * l[j];
                r[j] = rj;
                rr2 += rj * rj;
            }
            rr2 = block_sum1(rr2, sc);
            ++it;
            if (rr2 <= stop) break;
            const double beta = rr2 / rr;
            rr = rr2;
            for (int j = tid; j < m; j += nt)
                if (cut(j)) h[j] = r[j] + beta * h[j];
            __syncthreads();
        }
        for (int j = tid; j < m; j += nt)
            if (cut(j)) dy[j] += xv[j];
        __syncthreads();
        return it;
    }

    // Newton solve (A D^2 A^T) dy = w: rounds of PCG on the current FP64 residual rho,
    // dy += correction, rho = w - Q dy recomputed in FP64 (iterative refinement).
    // Inside the interior-point method (mu > 0) a round is good enough once the
    // complementarity perturbation it leaves, max_j z_j |(A_M^-1 rho)_j|, is at most
    // xi_tol * mu; standalone (mu = 0) once ||rho|| <= ref_tol ||w||. Rounds run in PT; when a
    // PT round fails to halve the error measure, or ref_max PT rounds do not reach the goal,
    // the solve switches to FP64 vectors (kept in the frame's global workspace) for up to
    // ref_max more rounds. A round that increases the error measure is undone.
    // Returns PCG iterations; refine_rounds counts the extra rounds, escal the switches;
    // resid2 = ||rho||^2 / ||w||^2. On return rho holds the final residual and, when mu > 0,
    // f64 holds A_M^-1 rho.
    LPD_INLINE int solve(double mu, int &refine_rounds, int &escal, double &resid2, bool &met, bool warm = false)
    {
        met = true;
        double nw2 = 0.0;
        for (int j = tid; j < m; j += nt) {
            const double wj = cut(j) ? w[j] : 0.0;
            const double d0 = warm && cut(j) ? dy[j] : 0.0;
            rho[j] = wj;
            dy[j] = d0;
            c64[7][j] = d0;
            nw2 += wj * wj;
        }
        nw2 = block_sum1(nw2, sc);
        resid2 = 0.0;
        if (!(nw2 > 0.0)) {
            for (int j = tid; j < m; j += nt) f64[j] = 0.0;
            __syncthreads();
            return 0;
        }
        if (warm && !(residual64() < nw2)) {
            // the previous Newton direction (the initial guess of Algorithm 4) is kept only
            // when it leaves a smaller residual than 0 does
            for (int j = tid; j < m; j += nt) {
                rho[j] = cut(j) ? w[j] : 0.0;
                dy[j] = 0.0;
                c64[7][j] = 0.0;
            }
            __syncthreads();
        }
        const bool use_xi = mu > 0.0;
        const double xi_goal = o.xi_tol * mu;
        CG<PT> V1 = {r, v, h, l, s, t, idm, om, d2f};
        CG<double> V2 = {c64[0], c64[1], c64[2], c64[3], st64, st64 + m, c64[5], c64[6], d2};
        const double tol1 = sizeof(PT) == 8 ? (o.ref_tol < o.pcg_tol ? o.ref_tol : o.pcg_tol) : o.pcg_tol;
        const double tol2 = o.ref_tol < o.pcg_tol ? o.ref_tol : o.pcg_tol;
        const double xs = use_xi ? xi_goal : 0.0;
        int its = 0, wide = sizeof(PT) == 8, left = o.ref_max;
        double prev = use_xi ? 1e300 : nw2;
        const int cap = pcg_cap();
        for (int rd = 0;; ++rd) {
            const int ri = o.precond == 4 ? plain_cg_round(tol2)
                                          : (wide && sizeof(PT) != 8 ? cg_round<double>(V2, tol2, xs) : cg_round<PT>(V1, tol1, xs));
            its += ri;
            double nr2 = residual64();
            double err = use_xi ? xi_max() : nr2;
            if (!(err < prev)) {
                // undo the round
                for (int j = tid; j < m; j += nt)
                    if (cut(j)) dy[j] = c64[7][j];
                __syncthreads();
                nr2 = residual64();
                err = use_xi ? xi_max() : nr2;
            }
            resid2 = nr2 / nw2;
            const bool done = use_xi ? (err <= xi_goal || nr2 <= o.ref_tol * o.ref_tol * nw2)
                                     : (nr2 <= o.ref_tol * o.ref_tol * nw2);
            met = done;
            if (done || !(err == err)) break;
            // a round that ran into the cap inside the IPM hands the system to the dense
            // solve, when there is one: refinement only pays after a PCG round that converged
            if (use_xi && qd && ri >= cap) break;
            if (!wide && (err > (use_xi ? 0.5 : 0.25) * prev || left <= 0)) {
                wide = 1;
                ++escal;
                left = o.ref_max;
            } else if (left-- <= 0) {
                break;
            }
            prev = err;
            for (int j = tid; j < m; j += nt) c64[7][j] = dy[j];   // kept for an undo
            __syncthreads();
            ++refine_rounds;
        }
        return its;
    }

    // ------------------------------------------------------------ dense fallback
    // The Newton matrix Q = A D^2 A^T over the LP rows (ascending check order) is padded to
    // Pp rows, a multiple of T = kDenseTile, with unit diagonal entries, and held row-major in
    // the frame's global workspace; only tiles on and below the diagonal are used (diagonal
    // tiles are read below their diagonal only). Blocked right-looking Cholesky: per block
    // column K, wave 0 factorises the diagonal tile in registers, every thread solves panel
    // rows against it, and the waves update the trailing lower tiles on the matrix cores.
    // Pivot rule: a pivot not above 1e-30 dm becomes 1e128.

    // Diagonal tile at (K, K), wave 0 only: lanes r and r + 32 both hold row r in registers
    // and compute the same values, so every LDS store of the loop is unconditional (equal
    // values to one address). Per pivot column c the lanes post their entry of the column to
    // LDS and read the pivot and the multipliers of the later rows back as broadcasts. Writes the factor back to Q with the
    // reciprocal of each diagonal entry in place of the entry (what the substitutions use),
    // and to LDS column-major (ldsd[c T + r] = L[r][c], c < r) with the reciprocals at
    // ldsd[T T + c].
    LPD_INLINE void dense_diag(double *Q, int Pp, int K, double dm)
    {
        constexpr int T = kDenseTile;
        const int lane = tid & 63, r = lane & (T - 1);
        double *const row = Q + (size_t)(K + r) * Pp + K;
        double *const colbuf = ldsd;   // column c of the tile before scaling, at colbuf[c T + r]
        double a[T];
#pragma unroll
        for (int c = 0; c < T; c += 2) {
            const double2 v = *(const double2 *)(row + c);
            a[c] = v.x;
            a[c + 1] = v.y;
        }
#pragma unroll
        for (int c = 0; c < T; ++c) {
            colbuf[c * T + r] = a[c];
            double s = colbuf[c * T + c];
            if (!(s > 1e-30 * dm)) s = 1e128;
            // 1/sqrt(s): the hardware estimate refined by two Newton steps y (3 - s y^2) / 2
            double inv = __builtin_amdgcn_rsq(s);
            inv = inv * (1.5 - 0.5 * s * inv * inv);
            inv = inv * (1.5 - 0.5 * s * inv * inv);
            a[c] = r == c ? inv : (r > c ? a[c] * inv : a[c]);
            ldsd[T * T + c] = inv;
            const double lrc = a[c];
#pragma unroll
            for (int cc = c + 1; cc < T; ++cc) a[cc] -= lrc * (colbuf[c * T + cc] * inv);
        }
        if (lane < T) {
#pragma unroll
            for (int c = 0; c < T; c += 2) *(double2 *)(row + c) = make_double2(a[c], a[c + 1]);
#pragma unroll
            for (int c = 0; c < T; ++c) ldsd[c * T + r] = a[c];
        }
        // forward substitution of this block (L y = colk, fused into the factorisation): the
        // rows below were already reduced by the earlier panels
        double v = colk[K + r];
#pragma unroll
        for (int c = 0; c < T; ++c) {
            const double xc = lp_readlane_d(v, c) * lp_readlane_d(a[c], c);
            v = r == c ? xc : (r > c ? v - a[c] * xc : v);
        }
        if (lane < T) {
            colk[K + r] = v;
            ldsd[T * T + T + r] = v;
        }
    }

    // Rows below the diagonal tile: row i becomes x with x L_KK^T = a_i, one thread per row,
    // the row in registers; each solved entry is subtracted from the later ones at once.
    LPD_INLINE void dense_panel(double *Q, int Pp, int K)
    {
        constexpr int T = kDenseTile;
        const double *const Lc = ldsd, *const dinv = ldsd + T * T;
        for (int i = K + T + tid; i < Pp; i += nt) {
            double *const row = Q + (size_t)i * Pp + K;
            // an opaque zero offset keeps the factor's LDS reads inside the loop (hoisted
            // out, they would need 528 registers)
            int o0 = 0;
            asm volatile("" : "+v"(o0));
            double a[T];
#pragma unroll
            for (int c = 0; c < T; c += 2) {
                const double2 v = *(const double2 *)(row + c);
                a[c] = v.x;
                a[c + 1] = v.y;
            }
#pragma unroll
            for (int c = 0; c < T; ++c) {
                a[c] *= dinv[o0 + c];
#pragma unroll
                for (int cc = c + 1; cc < T; ++cc) a[cc] -= a[c] * Lc[o0 + c * T + cc];
            }
#pragma unroll
            for (int c = 0; c < T; c += 2) *(double2 *)(row + c) = make_double2(a[c], a[c + 1]);
            // the fused forward substitution: this row's right-hand side loses L_iK y_K
            const double *const yk = ldsd + T * T + T;
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int c = 0; c < T; c += 2) {
                s0 += a[c] * yk[o0 + c];
                s1 += a[c + 1] * yk[o0 + c + 1];
            }
            colk[i] -= s0 + s1;
        }
    }

    // Trailing update C -= L_I L_J^T of every tile (I, J) on or below the diagonal right of
    // block column K. A 32 x 32 tile is 2 x 2 blocks of the FP64 16x16x4 matrix-core product:
    // lane l gives row (l mod 16) of a block at k-slot (l div 16) for both operands and
    // accumulates rows (l div 16) + 4 v, v = 0..3, of column (l mod 16). k-slot s of step t
    // is panel column 8 s + t, so each lane reads 8 consecutive entries of a row. A wave owns
    // whole tile rows (longest first, dealt in zig-zag order over the waves), keeps the row's
    // panel operand in registers and loads the next tile while the current one is computed.
    struct DTile {
        lp_d4 acc[2][2];
        double bv[2][8];
    };
    LPD_INLINE void dtile_load(const double *Q, int Pp, int K, int I0, int J0, int lr, int lk, DTile &t)
    {
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int sj = 0; sj < 2; ++sj)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    t.acc[si][sj][v] = Q[(size_t)(I0 + 16 * si + lk + 4 * v) * Pp + J0 + 16 * sj + lr];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double *const pb = Q + (size_t)(J0 + 16 * s + lr) * Pp + K + 8 * lk;
#pragma unroll
            for (int k = 0; k < 8; k += 2) {
                const double2 y = *(const double2 *)(pb + k);
                t.bv[s][k] = y.x;
                t.bv[s][k + 1] = y.y;
            }
        }
    }
    LPD_INLINE void dtile_finish(double *Q, int Pp, int I0, int J0, int lr, int lk, DTile &t,
                                 const double (&av)[2][8])
    {
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int si = 0; si < 2; ++si)
#pragma unroll
                for (int sj = 0; sj < 2; ++sj)
                    t.acc[si][sj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[si][k], t.bv[sj][k], t.acc[si][sj], 0, 0, 0);
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int sj = 0; sj < 2; ++sj)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Q[(size_t)(I0 + 16 * si + lk + 4 * v) * Pp + J0 + 16 * sj + lr] = t.acc[si][sj][v];
    }
    LPD_INLINE void dense_trailing(double *Q, int Pp, int K)
    {
        constexpr int T = kDenseTile;
        const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
        const int lr = lane & 15, lk = lane >> 4;
        const int R0 = K + T, nT = (Pp - R0) / T;
        for (int k = 0; k < nT; ++k) {
            const int z = k % (2 * nw);
            if ((z < nw ? z : 2 * nw - 1 - z) != wv) continue;
            const int tI = nT - 1 - k, I0 = R0 + tI * T;
            double av[2][8];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const double *const pa = Q + (size_t)(I0 + 16 * s + lr) * Pp + K + 8 * lk;
#pragma unroll
                for (int kk = 0; kk < 8; kk += 2) {
                    const double2 x = *(const double2 *)(pa + kk);
                    av[s][kk] = -x.x;
                    av[s][kk + 1] = -x.y;
                }
            }
            DTile t0, t1;
            dtile_load(Q, Pp, K, I0, R0, lr, lk, t0);
            for (int tJ = 0;;) {
                if (tJ + 1 <= tI) dtile_load(Q, Pp, K, I0, R0 + (tJ + 1) * T, lr, lk, t1);
                dtile_finish(Q, Pp, I0, R0 + tJ * T, lr, lk, t0, av);
                if (++tJ > tI) break;
                if (tJ + 1 <= tI) dtile_load(Q, Pp, K, I0, R0 + (tJ + 1) * T, lr, lk, t0);
                dtile_finish(Q, Pp, I0, R0 + tJ * T, lr, lk, t1, av);
                if (++tJ > tI) break;
            }
        }
    }

    // Cholesky factor of the padded Q in place (lower triangle), block column by block column,
    // with the forward substitution L y = colk carried along (colk becomes y).
    LPD_INLINE void dense_factor(double *Q, int Pp, double dm)
    {
        constexpr int T = kDenseTile;
        for (int K = 0; K < Pp; K += T) {
            if (tid < 64) dense_diag(Q, Pp, K, dm);
            __syncthreads();
            dense_panel(Q, Pp, K);
            __syncthreads();
            dense_trailing(Q, Pp, K);
            __syncthreads();
        }
    }

    // L^T x = y in place in colk (Pp entries; y comes from the forward substitution fused
    // into dense_factor) by blocks of T rows: wave 0 solves the diagonal block in registers,
    // the workgroup updates the other rows. The diagonal of Q holds the reciprocals of L's
    // diagonal.
    LPD_INLINE void dense_subst(const double *Q, int Pp)
    {
        constexpr int T = kDenseTile;
        double *const xs = ldsd + T * T + T;
        const int r = tid & (T - 1);
        double bn[T];   // wave 0: column r of the next diagonal block, loaded one block ahead
        if (tid < 64 && Pp >= T) {
#pragma unroll
            for (int c = 0; c < T; ++c) bn[c] = Q[(size_t)(Pp - T + c) * Pp + Pp - T + r];
        }
        for (int K = Pp - T; K >= 0; K -= T) {
            if (tid < 64) {
                const int lane = tid;
                double bc[T];   // bc[c] = L[K + c][K + r]
#pragma unroll
                for (int c = 0; c < T; ++c) bc[c] = bn[c];
                double v = colk[K + r];
#pragma unroll
                for (int c = T - 1; c >= 0; --c) {
                    const double xc = lp_readlane_d(v, c) * lp_readlane_d(bc[c], c);
                    v = lane == c ? xc : (lane < c ? v - bc[c] * xc : v);
                }
                if (lane < T) { colk[K + r] = v; xs[r] = v; }
            }
            __syncthreads();
            if (tid < 64 && K >= T) {
#pragma unroll
                for (int c = 0; c < T; ++c) bn[c] = Q[(size_t)(K - T + c) * Pp + K - T + r];
            }
            for (int j = tid; j < K; j += nt) {
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int c = 0; c < T; c += 2) {
                    s0 += Q[(size_t)(K + c) * Pp + j] * xs[c];
                    s1 += Q[(size_t)(K + c + 1) * Pp + j] * xs[c + 1];
                }
                colk[j] -= s0 + s1;
            }
            __syncthreads();
        }
    }

    // Dense fallback for a Newton system the PCG rounds did not finish: assembles Q, factorises
    // it, then forward and back substitution by blocks of T rows (wave 0 solves the diagonal
    // block in registers, the workgroup updates the rest). Writes dy; the caller recomputes
    // the FP64 residual. Returns the padded order Pp.
    LPD_INLINE int direct_solve()
    {
        constexpr int T = kDenseTile;
        for (int j = tid; j < m; j += nt) ridx[j] = cut(j) ? 1 : 0;
        block_exscan(ridx, m);
        const int P = ridx[m], Pp = (P + T - 1) / T * T;
        double *const Q = qd;
        // zero the tiles on and below the diagonal (the only ones read), a wave per row
        for (int rr = tid >> 6; rr < Pp; rr += nt >> 6) {
            double2 *const q2 = (double2 *)(Q + (size_t)rr * Pp);
            const int w2 = ((rr / T) + 1) * (T / 2);
            for (int c2 = tid & 63; c2 < w2; c2 += 64) q2[c2] = make_double2(0.0, 0.0);
        }
        __syncthreads();
        // lower triangle, one thread per LP row: row r gets a_ri a_r'i d_i^2 for every column i
        // of the row and every row r' <= r of that column, and the row's slack weight
        double dm = 0.0;
        for (int j = tid; j < m; j += nt) {
            if (!cut(j)) continue;
            const int r = ridx[j];
            double *const Qr = Q + (size_t)r * Pp;
            double diag = d2[n + j];
            for (int k = 0; k < RW; ++k) {
                const uint16_t e = rlist[(size_t)j * RW + k];
                if (e == kEnd) break;
                const int i = e_idx(e);
                const double di = d2[i];
                for (int q = 0; q < CW; ++q) {
                    const uint16_t e2 = clist[(size_t)i * CW + q];
                    if (e2 == kEnd) break;
                    const int j2 = e_idx(e2);
                    if (j2 == j) { diag += di; continue; }
                    const int r2 = ridx[j2];
                    if (r2 < r) Qr[r2] += (e_neg(e) != e_neg(e2) ? -di : di);
                }
            }
            Qr[r] = diag;
            dm = fmax(dm, diag);
        }
        for (int r = P + tid; r < Pp; r += nt) Q[(size_t)r * Pp + r] = 1.0;
        // right-hand side in colk, indexed by LP row (the padding rows are zero): the
        // factorisation also runs the forward substitution L y = w, then L^T x = y
        for (int j = tid; j < m; j += nt)
            if (cut(j)) colk[ridx[j]] = w[j];
        for (int r = P + tid; r < Pp; r += nt) colk[r] = 0.0;
        dm = block_max_d(dm, sc);
        dense_factor(Q, Pp, dm);
        dense_subst(Q, Pp);
        for (int j = tid; j < m; j += nt)
            if (cut(j)) dy[j] = colk[ridx[j]];
        __syncthreads();
        return Pp;
    }

    LPD_INLINE void set_d2f(int c, double dd)
    {
        const double vv = dd < 1e-30 ? 1e-30 : (dd > 1e30 ? 1e30 : dd);
        d2f[c] = (PT)vv;
    }

    // ------------------------------------------------------------ interior-point method
    // Infeasible primal-dual path-following method of Sec. IV-B on the LP of the current
    // cut set (rows = checks with a cut): residuals r_b = b - Ax, r_c = c - A^T y - z,
    // mu = sigma x^T z / q, r_e = mu e - XZe, D^2 = X Z^-1; Newton direction from
    // (A D^2 A^T) dy = r_b + A D^2 r_c - A Z^-1 r_e, dx = D^2 A^T dy - D^2 r_c + Z^-1 r_e,
    // dz = X^-1 (r_e - Z dx); separate primal and dual step lengths (fraction eta of the
    // distance to the boundary, at most 1). Starts at x = e, y = 0, z = e; stops when
    // x^T z / (1 + |c^T x|), ||r_b|| / (1 + ||b||) and ||r_c|| / (1 + ||c||) are all < eps,
    // or when the largest of them is below eps_stall and has not at least halved over the
    // last two iterations (the double-precision floor of a degenerate LP).
    // The LP's row and column lists must be built. Returns 0 or a negative LPDEC_FLAG_*.
    LPD_INLINE int ipm(lpdec_stats &st, int &iters)
    {
        double a0[2] = {0.0, 0.0};
        int pl = 0;
        // start point: x = e, y = 0, z = e; with IPM_WARM = theta > 0 an LP after the first
        // starts from the previous LP's point shifted into the interior (x + theta, z +
        // theta; y kept) on the columns and rows it shares with that LP (the method accepts
        // any x > 0, z > 0, Sec. IV-B)
        const double th = o.ipm_warm;
        const bool warm = th > 0.0 && have_prev;
        for (int j = tid; j < m; j += nt) {
            if (cut(j)) {
                // b of the flipped parity inequality: |V| - 1 - sum of its u-coefficients
                // over variables with sigma_i = -1
                const uint32_t V = vmask[j];
                const int e0 = cd.rowptr[j], e1 = cd.rowptr[j + 1];
                int vsz = 0, sneg = 0;
                for (int e = e0; e < e1; ++e) {
                    const int sv = ((V >> (e - e0)) & 1u) ? 1 : -1;
                    vsz += sv > 0;
                    if (sg[cd.col[e]] < 0) sneg += sv;
                }
                const double bj = (double)(vsz - 1 - sneg);
                b[j] = bj;
                a0[0] += bj * bj;
                if (warm && vprev[j] == V) {
                    x[n + j] += th; z[n + j] += th;
                } else {
                    x[n + j] = 1.0; z[n + j] = 1.0; y[j] = 0.0;
                }
                ++pl;
            } else {
                b[j] = 0.0; x[n + j] = 0.0; z[n + j] = 0.0; y[j] = 0.0;
            }
            vprev[j] = cut(j) ? vmask[j] : 0u;
        }
        for (int i = tid; i < n; i += nt) {
            if (warm) { x[i] += th; z[i] += th; }
            else { x[i] = 1.0; z[i] = 1.0; }
            a0[1] += g[i] * g[i];
        }
        block_sum<2>(a0, sc);
        p = block_sum1(pl, sc);
        const double nb = sqrt(a0[0]), nc = sqrt(a0[1]);
        const double q = (double)(n + p);
        int status = LPDEC_FLAG_IPM_CAP, it;
        double phi1 = INFINITY, phi2 = INFINITY;   // error measure one and two iterations ago
        // set once PCG has failed on this LP: its later Newton systems are only worse
        // conditioned, so they go straight to the dense solve
        bool direct_mode = false;
        for (it = 0; it < o.ipm_max; ++it) {
            double a[4] = {0.0, 0.0, 0.0, 0.0};   // gap, c^T x, ||r_b||^2, ||r_c||^2
            for (int j = tid; j < m; j += nt) {
                if (!cut(j)) continue;
                const double rbj = b[j] - row_dot<double>(j, x);
                rb[j] = rbj;
                a[2] += rbj * rbj;
            }
            for (int c = tid; c < n + m; c += nt) {
                if (!colpresent(c)) continue;
                const double aty = c < n ? col_dot<double>(c, y) : y[c - n];
                const double cc = cost(c);
                const double rcc = cc - aty - z[c];
                rc[c] = rcc;
                a[3] += rcc * rcc;
                a[0] += x[c] * z[c];
                a[1] += cc * x[c];
            }
            block_sum<4>(a, sc);
            if (!isfinite(a[0]) || !isfinite(a[1]) || !isfinite(a[2]) || !isfinite(a[3])) {
                status = LPDEC_FLAG_NONFINITE;
                break;
            }
            const double phi = fmax(a[0] / (1.0 + fabs(a[1])),
                                    fmax(sqrt(a[2]) / (1.0 + nb), sqrt(a[3]) / (1.0 + nc)));
            if (phi < o.eps || (phi < o.eps_stall && phi > 0.5 * phi2)) {
                status = 0;
                break;
            }
            phi2 = phi1;
            phi1 = phi;
            const double mu = o.sigma * a[0] / q;
            for (int c = tid; c < n + m; c += nt) {
                if (!colpresent(c)) continue;
                const double dd = x[c] / z[c];
                d2[c] = dd;
                set_d2f(c, dd);
                const double re = mu - x[c] * z[c];
                tq[c] = dd * rc[c] - re / z[c];
            }
            __syncthreads();
            for (int j = tid; j < m; j += nt)
                if (cut(j)) w[j] = rb[j] + row_dot<double>(j, tq);
            // preconditioner for this iteration. Sec. V-B searches it anew at every iteration;
            // with MTS_REUSE = R > 1 the set found on iteration it - (it mod R) of this LP is
            // kept (the weights d of the current iteration still enter through D_M), which is
            // the reuse across iterations that Sec. V-C leaves open
            const long long t0 = wall_clock64();
            const bool search = it % o.mts_reuse == 0;
            int tri_calls = 0;
            if (!direct_mode && search) {
                tri_calls = find_precond_set();
                build_levels();
                st.max_levels = max(st.max_levels, max(nlb, nlf));
            }
            const long long t1 = wall_clock64();
            double resid2 = 0.0;
            bool met = true;
            const int pits = direct_mode ? 0 : solve(mu, st.ref_rounds, st.escalations, resid2, met, o.warm && it > 0);
            if ((direct_mode || !met) && qd) {
                // PCG did not reach the goal (now or earlier in this LP): the Newton system is
                // solved directly; its residual is at rounding level, so the completion below
                // gets no correction term
                const long long td = wall_clock64();
                const long long pp = direct_solve();
                for (int j = tid; j < m; j += nt) f64[j] = 0.0;
                __syncthreads();
                ++st.direct_solves;
                st.ticks_dense += wall_clock64() - td;
                st.dense_cube += pp * pp * pp;
                direct_mode = true;
            }
            const long long t2 = wall_clock64();
            st.ticks_mts += t1 - t0;
            st.ticks_solve += t2 - t1;
            st.mts_rounds += o.precond && !direct_mode && search ? (o.precond == 5 ? tri_calls : p) : 0;
            st.pcg_iters += pits;
            st.pcg_rows += (long long)pits * p;
            st.ipm_cols += n + p;
            // Newton completion. With an exact dy this is dx = D^2 A^T dy - D^2 r_c + Z^-1 r_e,
            // dz = X^-1 (r_e - Z dx) = r_c - A^T dy. The residual rho = w - Q dy of the
            // iterative solve is moved into the complementarity equation: dx gets
            // delta = A_M^-1 rho (left in f64 by the solve) on the preconditioning set, so
            // A dx = r_b and A^T dy + dz = r_c hold exactly and Z dx + X dz = r_e + Z delta.
            double bp = 1e300, bd = 1e300;
            for (int c = tid; c < n + m; c += nt) {
                if (!colpresent(c)) continue;
                const double aty = c < n ? col_dot<double>(c, dy) : dy[c - n];
                const double dd = d2[c];
                const double re = mu - x[c] * z[c];
                double dxc = dd * (aty - rc[c]) + re / z[c];
                if (c < n) { if (pairrow[c] >= 0) dxc += f64[pairrow[c]]; }
                else if (pair[c - n] == c) dxc += f64[c - n];
                const double dzc = rc[c] - aty;
                dx[c] = dxc;
                dz[c] = dzc;
                if (dxc < 0.0) bp = fmin(bp, -x[c] / dxc);
                if (dzc < 0.0) bd = fmin(bd, -z[c] / dzc);
            }
            block_min2(bp, bd, sc);
            bp = fmin(1.0, o.eta * bp);
            bd = fmin(1.0, o.eta * bd);
            for (int c = tid; c < n + m; c += nt) {
                if (!colpresent(c)) continue;
                x[c] += bp * dx[c];
                z[c] += bd * dz[c];
            }
            for (int j = tid; j < m; j += nt)
                if (cut(j)) y[j] += bd * dy[j];
            __syncthreads();
        }
        iters = it;
        return status;
    }

    // ------------------------------------------------------------ MALP decoding
    LPD_INLINE void load_gamma(const Args &a, int f)
    {
        for (int i = tid; i < n; i += nt) {
            const size_t k = (size_t)f * n + i;
            const double gi = a.gamma_f64 ? ((const double *)a.gamma)[k] : (double)((const float *)a.gamma)[k];
            g[i] = gi;
            sg[i] = gi >= 0.0 ? 1 : -1;
        }
    }

    // Algorithm 3 (MALP-A) or MALP-B, then the output decisions.
    LPD_INLINE void decode(const Args &a, int f)
    {
        lpdec_stats st = {};
        ticks_pcg = 0;
        const long long t_start = wall_clock64();
        load_gamma(a, f);
        double gneg = 0.0;   // gamma^T u at the hard decision
        for (int i = tid; i < n; i += nt) {
            u[i] = g[i] >= 0.0 ? 0.0 : 1.0;   // hard decision
            if (g[i] < 0.0) gneg += g[i];
        }
        for (int j = tid; j < m; j += nt) { vmask[j] = 0u; active[j] = 0; vprev[j] = 0u; vback[j] = 0u; }
        have_prev = false;
        gneg = block_sum1(gneg, sc);
        double cost_prev = gneg;    // gamma^T u of the previous LP's solution
        double cost_prev2 = gneg;   // and of the one before
        bool last = false;          // the LP about to be solved ends the decode
        int status = 0, k;
        for (k = 0; k < o.malp_max; ++k) {
            int added = 0;
            for (int j = tid; j < m; j += nt) {
                if (o.malp_mode == 1 && vmask[j] && !active[j]) vmask[j] = 0u;
                if (vmask[j] && active[j]) continue;   // a check with an active cut is skipped
                uint32_t V;
                double lhs;
                if (find_cut(j, V, lhs)) { vmask[j] = V; active[j] = 0; added = 1; }
            }
            added = block_or(added, sc);
            if (!added) break;
            // A cut set equal to that of two LPs back contradicts Theorem 2b; it comes from an
            // optimum that is not unique at the IPM's accuracy, where a cut that bounds the
            // optimum looks inactive. The steps are deterministic, so the two LPs would
            // alternate until the cap: the decode ends with the solution of the costlier one,
            // u^(k-1) as it stands or this LP (the same as LP k-2) solved once more.
            if (k >= 2) {
                int diff = 0;
                for (int j = tid; j < m; j += nt) diff |= vmask[j] != vback[j];
                if (!block_or(diff, sc)) {
                    if (cost_prev >= cost_prev2) { status = LPDEC_FLAG_CUT_CYCLE; break; }
                    last = true;
                }
            }
            // vprev holds LP k-1's cuts until ipm() records this LP's
            for (int j = tid; j < m; j += nt) vback[j] = vprev[j];
            if (a.trace && k < a.trace_cap)
                for (int j = tid; j < m; j += nt) a.trace[((size_t)f * a.trace_cap + k) * m + j] = vmask[j];
            build_lists();
            int its = 0;
            status = ipm(st, its);
            have_prev = status >= 0;
            st.malp_iters++;
            st.ipm_iters += its;
            st.p_max = max(st.p_max, p);
            // u^k from the LP solution, put back on the box [0, 1]^n that every u^k satisfies
            // (Theorem 2a): a coordinate of tiny cost that the gap test leaves slightly
            // outside would otherwise let Algorithm 2 report a violated cut from rounding
            double cost = 0.0;
            for (int i = tid; i < n; i += nt) {
                const double ui = fmin(1.0, fmax(0.0, sg[i] > 0 ? x[i] : 1.0 - x[i]));
                u[i] = ui;
                cost += g[i] * ui;
            }
            for (int j = tid; j < m; j += nt) {
                if (!cut(j)) { active[j] = 0; continue; }
                const double sl = x[n + j], zs = z[n + j];
                active[j] = !(sl > (o.tau_act > zs ? o.tau_act : zs));
            }
            cost = block_sum1(cost, sc);
            if (status < 0) break;
            if (last) { status = LPDEC_FLAG_CUT_CYCLE; break; }
            // Theorem 2b: successive LP costs increase strictly. A decrease beyond the IPM's
            // accuracy (relative to 1 + c^T x, c^T x = gamma^T u - gneg) means a cut that still
            // bound the optimum was replaced or dropped; the decode ends with a failure flag
            if (cost < cost_prev - o.tau_cost * (1.0 + fabs(cost_prev - gneg))) {
                status = LPDEC_FLAG_COST_DECREASE;
                break;
            }
            cost_prev2 = cost_prev;
            cost_prev = cost;
        }
        if (k == o.malp_max && status == 0) status = LPDEC_FLAG_MALP_CAP;
        // output: integrality, decisions, syndrome, objective gamma^T u
        double fr = 0.0, ob = 0.0;
        for (int i = tid; i < n; i += nt) {
            const double ui = u[i];
            const double d = ui < 1.0 - ui ? ui : 1.0 - ui;
            fr = d > fr ? d : fr;
            ob += g[i] * ui;
            const int xh = fabs(ui - 0.5) <= o.tau_int ? (g[i] >= 0.0 ? 0 : 1) : (ui > 0.5 ? 1 : 0);
            deg[i] = (uint8_t)xh;   // the decisions, kept for the syndrome
            a.xhat[(size_t)f * n + i] = (uint8_t)xh;
            if (a.u_out) a.u_out[(size_t)f * n + i] = ui;
        }
        fr = block_max_d(fr, sc);
        ob = block_sum1(ob, sc);
        int syn = 0;
        for (int j = tid; j < m; j += nt) {
            int par = 0;
            for (int e = cd.rowptr[j]; e < cd.rowptr[j + 1]; ++e) par ^= deg[cd.col[e]];
            syn |= par;
        }
        syn = block_or(syn, sc);
        if (tid == 0) {
            int flag;
            if (status < 0) flag = status;
            else if (fr <= o.tau_int && !syn) flag = 1;
            else if (fr <= o.tau_int) flag = LPDEC_FLAG_INCONSISTENT;
            else flag = 0;
            a.flag[f] = flag;
            if (a.obj) a.obj[f] = ob;
            st.status = status;
            st.ticks_total = wall_clock64() - t_start;
            st.ticks_pcg = ticks_pcg;
            if (a.stats) a.stats[f] = st;
        }
        if (a.done) {
            // every thread's output stores reach the system before the frame is marked done
            __threadfence_system();
            __syncthreads();
            if (tid == 0) __hip_atomic_store(&a.done[f], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
};

}  // namespace lpdec
