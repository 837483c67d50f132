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
    unsigned long long *lbest;
    uint32_t *ldirty;
    // cold
    double *x, *z, *dx, *dz, *rc, *tq, *d2, *y, *dy, *rb, *w, *b, *rho, *f64, *u, *g;
    double *c64[8];   // FP64 PCG vectors for escalated solves, and a copy of dy
    uint8_t *active;
    // level counts of the current preconditioner, LP rows
    int nlb, nlf, p;

    LPD_INLINE void bind(const Args &a, char *hot, char *cold, Scratch *scr)
    {
        cd = a.code; o = a.o; m = cd.m; n = cd.n; RW = cd.dcmax; CW = cd.dvmax;
        tid = threadIdx.x; nt = blockDim.x; sc = scr;
        const Plan &P = a.plan;
        h = (PT *)(hot + P.h); r = (PT *)(hot + P.r); v = (PT *)(hot + P.v); l = (PT *)(hot + P.l);
        s = (PT *)(hot + P.s); idm = (PT *)(hot + P.idm); om = (PT *)(hot + P.om);
        t = (PT *)(hot + P.t); d2f = (PT *)(hot + P.d2f);
        rlist = (uint16_t *)(hot + P.rlist); clist = (uint16_t *)(hot + P.clist);
        bins = (uint16_t *)(hot + P.bins); fins = (uint16_t *)(hot + P.fins);
        pair = (int16_t *)(hot + P.pair); pairrow = (int16_t *)(hot + P.pairrow);
        lbv = (int16_t *)(hot + P.lbv); lfv = (int16_t *)(hot + P.lfv); order = (int16_t *)(hot + P.order);
        boff = (int *)(hot + P.boff); foff = (int *)(hot + P.foff);
        deg = (uint8_t *)(hot + P.deg); sg = (int8_t *)(hot + P.sg); vmask = (uint32_t *)(hot + P.vmask);
        lbest = (unsigned long long *)(hot + P.lbest); ldirty = (uint32_t *)(hot + P.ldirty);
        x = (double *)(cold + P.x); z = (double *)(cold + P.z); dx = (double *)(cold + P.dx);
        dz = (double *)(cold + P.dz); rc = (double *)(cold + P.rc); tq = (double *)(cold + P.tq);
        d2 = (double *)(cold + P.d2); y = (double *)(cold + P.y); dy = (double *)(cold + P.dy);
        rb = (double *)(cold + P.rb); w = (double *)(cold + P.w); b = (double *)(cold + P.b);
        rho = (double *)(cold + P.rho); f64 = (double *)(cold + P.f64);
        u = (double *)(cold + P.u); g = (double *)(cold + P.g);
        for (int k = 0; k < 8; ++k) c64[k] = (double *)(cold + P.c64 + (size_t)k * lp_align(8 * (size_t)m));
        active = (uint8_t *)(cold + P.active);
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
        const uint16_t *L = rlist + (size_t)j * RW;
        T acc = (T)xq[n + j];
        for (int k = 0; k < RW; ++k) {
            const uint16_t e = L[k];
            if (e == kEnd) break;
            acc += sgnv(e, (T)xq[e_idx(e)]);
        }
        return acc;
    }
    // (A^T y)_i for standard column i, y in check space
    template <typename T, typename V>
    LPD_INLINE T col_dot(int i, const V *yy) const
    {
        const uint16_t *L = clist + (size_t)i * CW;
        T acc = 0;
        for (int k = 0; k < CW; ++k) {
            const uint16_t e = L[k];
            if (e == kEnd) break;
            acc += sgnv(e, (T)yy[e_idx(e)]);
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

    // preferred available column among those owned by one lane (c = lane + 64 k)
    LPD_INLINE unsigned long long lane_best(const float *wk, int lane) const
    {
        unsigned long long best = 0ull;
        for (int c = lane; c < n + m; c += 64) {
            bool av;
            if (c < n) av = pairrow[c] < 0 && deg[c] == 1;
            else av = cut(c - n) && pair[c - n] < 0;
            if (av) {
                const unsigned long long k = mts_key(wt(wk, c), c);
                best = k > best ? k : best;
            }
        }
        return best;
    }

    // Column-wise greedy search for the triangular set (Algorithm 7), exactly as stated:
    // p times, take the degree-1 column with the largest key (weight, then lowest index)
    // and eliminate the only row it still has. Wave 0 runs it: every lane keeps the best
    // available column of the columns it owns (lbest), the wave takes the maximum, and the
    // lanes of the eliminated row update the residual degrees of its columns. A lane whose
    // best column was taken or lost its last row rescans its columns.
    // Fills pair (column of each row), pairrow (row of each chosen standard column), order
    // (rows in elimination order), lfv (forward-substitution level) and lbv
    // (back-substitution level). Returns p.
    LPD_INLINE int mts(const float *wk)
    {
        for (int i = tid; i < n; i += nt) {
            const uint16_t *L = clist + (size_t)i * CW;
            int dg = 0;
            for (int k = 0; k < CW && L[k] != kEnd; ++k) ++dg;
            deg[i] = (uint8_t)dg;
            pairrow[i] = -1;
        }
        int pl = 0;
        for (int j = tid; j < m; j += nt) {
            pair[j] = -1; lfv[j] = -1; lbv[j] = -1;
            pl += cut(j);
        }
        pl = block_sum1(pl, sc);
        p = pl;
        if (tid < 64) {
            const int lane = tid;
            lbest[lane] = lane_best(wk, lane);
            ldirty[lane] = 0;
            for (int step = 0; step < pl; ++step) {
                __builtin_amdgcn_wave_barrier();
                unsigned long long mine = lbest[lane];
                if (ldirty[lane]) {
                    mine = lane_best(wk, lane);
                    lbest[lane] = mine;
                    ldirty[lane] = 0;
                }
                const unsigned long long K = wave_max_u64(mine);
                if (K == 0ull) break;   // no degree-1 column: cannot happen while rows remain
                const int c = mts_key_col(K);
                // the row of c: its only live row; the other rows give the forward level
                int row, L = 0;
                if (c >= n) {
                    row = c - n;
                } else {
                    row = -1;
                    const uint16_t *CL = clist + (size_t)c * CW;
                    for (int k = 0; k < CW; ++k) {
                        const uint16_t e = CL[k];
                        if (e == kEnd) break;
                        const int j = e_idx(e);
                        if (pair[j] < 0) row = j;
                        else L = max(L, (int)lfv[j] + 1);
                    }
                    if (row < 0) break;   // a degree-1 column always has its live row
                }
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) {
                    pair[row] = (int16_t)c;
                    lfv[row] = (int16_t)L;
                    order[step] = (int16_t)row;
                    if (c < n) pairrow[c] = (int16_t)row;
                    ldirty[c & 63] = 1;
                    ldirty[(n + row) & 63] = 1;
                }
                __builtin_amdgcn_wave_barrier();
                // eliminate the row: its waiting columns lose one degree
                if (lane < RW) {
                    const uint16_t e = rlist[(size_t)row * RW + lane];
                    if (e != kEnd) {
                        const int i = e_idx(e);
                        if (i != c && pairrow[i] < 0) {
                            const int dgi = deg[i] - 1;
                            deg[i] = (uint8_t)dgi;
                            if (dgi == 1) atomicMax(&lbest[i & 63], mts_key(wt(wk, i), i));
                            else if (dgi == 0) ldirty[i & 63] = 1;
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            // back-substitution levels, rows in reverse elimination order: a row depends on
            // the rows of the other chosen columns in it, all eliminated later
            for (int step = pl - 1; step >= 0; --step) {
                const int row = order[step], c = pair[row];
                int L = 0;
                if (lane < RW) {
                    const uint16_t e = rlist[(size_t)row * RW + lane];
                    if (e != kEnd) {
                        const int i = e_idx(e);
                        if (i != c && pairrow[i] >= 0) L = lbv[pairrow[i]] + 1;
                    }
                }
                L = (int)wave_max_u32((uint32_t)L);
                if (lane == 0) lbv[row] = (int16_t)L;
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        return pl;
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
    // slots [L ? boff[L-1] : 0, boff[L]) of bins (RW+1 entries per slot), forward level L
    // slots [L ? foff[L-1] : 0, foff[L]) of fins (CW entries per slot). Slot header: the row
    // and the sign of its diagonal entry. Back entries: the other M-columns of the row as
    // references to their rows (coefficient negated), the columns outside M (the slack
    // included) as column references. Forward entries: the other rows of the paired column
    // (coefficient negated).
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
                uint16_t *B = bins + (size_t)atomicAdd(&boff[lbv[j]], 1) * (RW + 1);
                const uint16_t *L = rlist + (size_t)j * RW;
                bool dneg = false;
                int q = 1;
                for (int k = 0; k < RW; ++k) {
                    const uint16_t e = L[k];
                    if (e == kEnd) break;
                    const int i = e_idx(e);
                    if (i == c) { dneg = e_neg(e); continue; }
                    if (pairrow[i] >= 0) B[q++] = enc(pairrow[i], !e_neg(e), true);
                    else B[q++] = enc(i, e_neg(e), false);
                }
                if (c != n + j) B[q++] = enc(n + j, false, false);
                for (; q <= RW; ++q) B[q] = kEnd;
                B[0] = enc(j, dneg, false);
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
                        F[q++] = enc(jj, !e_neg(e), true);
                    }
                }
                for (; q < CW; ++q) F[q] = kEnd;
                F[0] = enc(j, dneg, false);
            }
        }
        __syncthreads();
    }

    // ------------------------------------------------------------ triangular solves
    // The preconditioning set M pairs every LP row j with one column pair[j]; A_M (rows by
    // paired columns) is triangular after permutation with entries +-1 (Sec. V). Vectors over
    // M's columns are stored at the row each column is paired with.
    // Back-substitution out = A_M^-1 u (levels ascending).
    template <typename T, typename UF>
    LPD_INLINE void back_sub(T *out, UF u_of_row)
    {
        for (int L = 0; L < nlb; ++L) {
            const int k1 = boff[L];
            for (int k = (L ? boff[L - 1] : 0) + tid; k < k1; k += nt) {
                const uint16_t *B = bins + (size_t)k * (RW + 1);
                const uint16_t hd = B[0];
                const int j = e_idx(hd);
                T acc = u_of_row(j);
                for (int q = 1; q <= RW; ++q) {
                    const uint16_t e = B[q];
                    if (e == kEnd) break;
                    if (e_row(e)) acc += sgnv(e, out[e_idx(e)]);
                }
                out[j] = e_neg(hd) ? -acc : acc;
            }
            __syncthreads();
        }
    }

    // Forward substitution out = A_M^-T e (out in row space; levels ascending).
    template <typename T, typename EF>
    LPD_INLINE void fwd_sub(T *out, EF e_of_row)
    {
        for (int L = 0; L < nlf; ++L) {
            const int k1 = foff[L];
            for (int k = (L ? foff[L - 1] : 0) + tid; k < k1; k += nt) {
                const uint16_t *F = fins + (size_t)k * CW;
                const uint16_t hd = F[0];
                const int j = e_idx(hd);
                T acc = e_of_row(j);
                for (int q = 1; q < CW; ++q) {
                    const uint16_t e = F[q];
                    if (e == kEnd) break;
                    acc += sgnv(e, out[e_idx(e)]);
                }
                out[j] = e_neg(hd) ? -acc : acc;
            }
            __syncthreads();
        }
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
        T rr = 0;
        for (int j = tid; j < m; j += nt) { V.h[j] = V.r[j]; rr += V.r[j] * V.r[j]; }
        rr = block_sum1(rr, sc);
        if (!(rr > (T)0)) return 0;
        const T stop = tol * tol * rr;
        int it = 0;
        while (it < maxit) {
            // s = A_M^-T (D_M^-1 h)
            fwd_sub<T>(V.s, [&](int j) { return V.h[j] * V.idm[j]; });
            // t = D_N^2 A_N^T s on the columns outside M
            for (int c = tid; c < n + m; c += nt) {
                if (c < n) {
                    if (pairrow[c] < 0) V.t[c] = V.dsq[c] * col_dot<T>(c, V.s);
                } else {
                    const int j = c - n;
                    if (cut(j) && pair[j] != c) V.t[c] = V.dsq[c] * V.s[j];
                }
            }
            __syncthreads();
            // f = A_M^-1 (A_N t) over s; l = h + D_M^-1 f
            T hl = 0;
            for (int L = 0; L < nlb; ++L) {
                const int k1 = boff[L];
                for (int k = (L ? boff[L - 1] : 0) + tid; k < k1; k += nt) {
                    const uint16_t *B = bins + (size_t)k * (RW + 1);
                    const uint16_t hd = B[0];
                    const int j = e_idx(hd);
                    T acc = 0;
                    for (int q = 1; q <= RW; ++q) {
                        const uint16_t e = B[q];
                        if (e == kEnd) break;
                        acc += sgnv(e, e_row(e) ? V.s[e_idx(e)] : V.t[e_idx(e)]);
                    }
                    const T fj = e_neg(hd) ? -acc : acc;
                    V.s[j] = fj;
                    const T lj = V.h[j] + fj * V.idm[j];
                    V.l[j] = lj;
                    hl += V.h[j] * lj;
                }
                __syncthreads();
            }
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
        const int its = pcg<T>(V, (T)tol, (T)xi_stop, o.pcg_maxit);
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
            const uint16_t *L = rlist + (size_t)j * RW;
            double acc = d2[n + j] * dy[j];
            for (int k = 0; k < RW; ++k) {
                const uint16_t e = L[k];
                if (e == kEnd) break;
                acc += sgnv(e, tq[e_idx(e)]);
            }
            const double rj = w[j] - acc;
            rho[j] = rj;
            nr2 += rj * rj;
        }
        return block_sum1(nr2, sc);
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
    LPD_INLINE int solve(double mu, int &refine_rounds, int &escal, double &resid2)
    {
        double nw2 = 0.0;
        for (int j = tid; j < m; j += nt) {
            const double wj = cut(j) ? w[j] : 0.0;
            rho[j] = wj;
            dy[j] = 0.0;
            c64[7][j] = 0.0;
            nw2 += wj * wj;
        }
        nw2 = block_sum1(nw2, sc);
        resid2 = 0.0;
        if (!(nw2 > 0.0)) {
            for (int j = tid; j < m; j += nt) f64[j] = 0.0;
            __syncthreads();
            return 0;
        }
        const bool use_xi = mu > 0.0;
        const double xi_goal = o.xi_tol * mu;
        CG<PT> V1 = {r, v, h, l, s, t, idm, om, d2f};
        CG<double> V2 = {c64[0], c64[1], c64[2], c64[3], c64[4], tq, c64[5], c64[6], d2};
        const double tol1 = sizeof(PT) == 8 ? (o.ref_tol < o.pcg_tol ? o.ref_tol : o.pcg_tol) : o.pcg_tol;
        const double tol2 = o.ref_tol < o.pcg_tol ? o.ref_tol : o.pcg_tol;
        const double xs = use_xi ? xi_goal : 0.0;
        int its = 0, wide = sizeof(PT) == 8, left = o.ref_max;
        double prev = use_xi ? 1e300 : nw2;
        for (int rd = 0;; ++rd) {
            its += wide && sizeof(PT) != 8 ? cg_round<double>(V2, tol2, xs) : cg_round<PT>(V1, tol1, xs);
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
            if (done || !(err == err)) break;
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
    // x^T z / (1 + |c^T x|), ||r_b|| / (1 + ||b||) and ||r_c|| / (1 + ||c||) are all < eps.
    // The LP's row and column lists must be built. Returns 0 or a negative LPDEC_FLAG_*.
    LPD_INLINE int ipm(lpdec_stats &st, int &iters)
    {
        double a0[2] = {0.0, 0.0};
        int pl = 0;
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
                x[n + j] = 1.0; z[n + j] = 1.0;
                ++pl;
            } else {
                b[j] = 0.0; x[n + j] = 0.0; z[n + j] = 0.0;
            }
            y[j] = 0.0;
        }
        for (int i = tid; i < n; i += nt) {
            x[i] = 1.0; z[i] = 1.0;
            a0[1] += g[i] * g[i];
        }
        block_sum<2>(a0, sc);
        p = block_sum1(pl, sc);
        const double nb = sqrt(a0[0]), nc = sqrt(a0[1]);
        const double q = (double)(n + p);
        int status = LPDEC_FLAG_IPM_CAP, it;
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
            if (a[0] / (1.0 + fabs(a[1])) < o.eps && sqrt(a[2]) / (1.0 + nb) < o.eps &&
                sqrt(a[3]) / (1.0 + nc) < o.eps) {
                status = 0;
                break;
            }
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
            // preconditioner for this iteration (Sec. V-B: found anew at every iteration)
            const long long t0 = wall_clock64();
            if (o.precond) mts(nullptr);
            else slack_basis();
            build_levels();
            st.max_levels = max(st.max_levels, max(nlb, nlf));
            const long long t1 = wall_clock64();
            double resid2;
            const int pits = solve(mu, st.ref_rounds, st.escalations, resid2);
            const long long t2 = wall_clock64();
            st.ticks_mts += t1 - t0;
            st.ticks_solve += t2 - t1;
            st.mts_rounds += o.precond ? p : 0;
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
        const long long t_start = wall_clock64();
        load_gamma(a, f);
        for (int i = tid; i < n; i += nt) u[i] = g[i] >= 0.0 ? 0.0 : 1.0;   // hard decision
        for (int j = tid; j < m; j += nt) { vmask[j] = 0u; active[j] = 0; }
        __syncthreads();
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
            if (a.trace && k < a.trace_cap)
                for (int j = tid; j < m; j += nt) a.trace[((size_t)f * a.trace_cap + k) * m + j] = vmask[j];
            build_lists();
            int its = 0;
            status = ipm(st, its);
            st.malp_iters++;
            st.ipm_iters += its;
            st.p_max = max(st.p_max, p);
            for (int i = tid; i < n; i += nt) u[i] = sg[i] > 0 ? x[i] : 1.0 - x[i];
            for (int j = tid; j < m; j += nt) {
                if (!cut(j)) { active[j] = 0; continue; }
                const double sl = x[n + j], zs = z[n + j];
                active[j] = !(sl > (o.tau_act > zs ? o.tau_act : zs));
            }
            __syncthreads();
            if (status < 0) break;
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
            if (a.stats) a.stats[f] = st;
        }
    }
};

}  // namespace lpdec
