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
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lpdec_common.hpp"

namespace lpdec {

#define LPD_INLINE __device__ __forceinline__

constexpr int kMaxWaves = 16;   // up to 1024 threads per frame

// -------------------------------------------------------------------- block primitives
template <typename T>
LPD_INLINE T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T>
LPD_INLINE T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

template <typename T>
LPD_INLINE T wave_min(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

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
    T *buf = reinterpret_cast<T *>(s->d);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
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
}

template <typename T>
LPD_INLINE T block_sum1(T v, Scratch *s)
{
    T a[1] = {v};
    block_sum<1>(a, s);
    return a[0];
}

// [0] summed, [1] maximised over the block.
template <typename T>
LPD_INLINE void block_summax(T (&v)[2], Scratch *s)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    T *buf = reinterpret_cast<T *>(s->d);
    v[0] = wave_sum(v[0]);
    v[1] = wave_max(v[1]);
    __syncthreads();
    if (lane == 0) { buf[wv] = v[0]; buf[kMaxWaves + wv] = v[1]; }
    __syncthreads();
    T a = 0, b = buf[kMaxWaves];
    for (int w = 0; w < nw; ++w) {
        a += buf[w];
        b = buf[kMaxWaves + w] > b ? buf[kMaxWaves + w] : b;
    }
    v[0] = a;
    v[1] = b;
}

LPD_INLINE double block_max_d(double v, Scratch *s)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) s->d[wv] = v;
    __syncthreads();
    double a = s->d[0];
    for (int w = 1; w < nw; ++w) a = s->d[w] > a ? s->d[w] : a;
    return a;
}

LPD_INLINE void block_min2(double &a, double &b, Scratch *s)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    a = wave_min(a);
    b = wave_min(b);
    __syncthreads();
    if (lane == 0) { s->d[wv] = a; s->d[kMaxWaves + wv] = b; }
    __syncthreads();
    a = s->d[0];
    b = s->d[kMaxWaves];
    for (int w = 1; w < nw; ++w) {
        a = s->d[w] < a ? s->d[w] : a;
        b = s->d[kMaxWaves + w] < b ? s->d[kMaxWaves + w] : b;
    }
}

LPD_INLINE int block_or(int v, Scratch *s)
{
    const unsigned long long bal = __ballot(v != 0);
    __syncthreads();
    if (threadIdx.x == 0) s->i[0] = 0;
    __syncthreads();
    if ((threadIdx.x & 63) == 0 && bal) atomicOr(&s->i[0], 1);
    __syncthreads();
    return s->i[0];
}

LPD_INLINE int block_max_i(int v, Scratch *s)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) reinterpret_cast<int *>(s->d)[wv] = v;
    __syncthreads();
    int a = reinterpret_cast<int *>(s->d)[0];
    for (int w = 1; w < nw; ++w) {
        int b = reinterpret_cast<int *>(s->d)[w];
        a = b > a ? b : a;
    }
    return a;
}

// Exclusive scan over cnt[0..len) in place (one wave does it, chunks of 64); the others wait.
LPD_INLINE void block_exscan(int *cnt, int len)
{
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int carry = 0;
        for (int base = 0; base < len; base += 64) {
            int v = (base + lane < len) ? cnt[base + lane] : 0;
            int incl = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                int t = __shfl_up(incl, o, 64);
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
// packed so that a larger 64-bit integer means "preferred".
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
    int m, n, tid, nt;
    Scratch *sc;
    // hot
    PT *h, *r, *zz, *l, *yv, *t, *d2f, *idm, *om;
    uint32_t *vmask;
    int8_t *sg;
    int *pair, *pairrow, *rnd, *lb, *lf, *blist, *flist, *boff, *foff;
    unsigned long long *killkey;
    int *status;
    // cold
    double *x, *z, *dx, *dz, *rc, *tq, *d2, *y, *dy, *rb, *w, *b, *rho, *u, *g, *f64;
    double *c64[8];   // FP64 PCG vectors for escalated solves, and a copy of dy
    uint8_t *active;
    // level counts of the current preconditioner
    int nlb, nlf, p;

    LPD_INLINE void bind(const Args &a, char *hot, char *cold, Scratch *s)
    {
        cd = a.code; o = a.o; m = cd.m; n = cd.n; tid = threadIdx.x; nt = blockDim.x; sc = s;
        const Plan &P = a.plan;
        h = (PT *)(hot + P.h); r = (PT *)(hot + P.r); zz = (PT *)(hot + P.zz); l = (PT *)(hot + P.l);
        yv = (PT *)(hot + P.yv); t = (PT *)(hot + P.t); d2f = (PT *)(hot + P.d2f); idm = (PT *)(hot + P.idm); om = (PT *)(hot + P.om);
        vmask = (uint32_t *)(hot + P.vmask); sg = (int8_t *)(hot + P.sg);
        pair = (int *)(hot + P.pair); pairrow = (int *)(hot + P.pairrow); rnd = (int *)(hot + P.rnd);
        lb = (int *)(hot + P.lb); lf = (int *)(hot + P.lf); blist = (int *)(hot + P.blist);
        flist = (int *)(hot + P.flist); boff = (int *)(hot + P.boff); foff = (int *)(hot + P.foff);
        killkey = (unsigned long long *)(hot + P.killkey); status = (int *)(hot + P.status);
        x = (double *)(cold + P.x); z = (double *)(cold + P.z); dx = (double *)(cold + P.dx);
        dz = (double *)(cold + P.dz); rc = (double *)(cold + P.rc); tq = (double *)(cold + P.tq);
        d2 = (double *)(cold + P.d2); y = (double *)(cold + P.y); dy = (double *)(cold + P.dy);
        rb = (double *)(cold + P.rb); w = (double *)(cold + P.w); b = (double *)(cold + P.b);
        rho = (double *)(cold + P.rho); u = (double *)(cold + P.u); g = (double *)(cold + P.g);
        f64 = (double *)(cold + P.f64);
        for (int k = 0; k < 8; ++k) c64[k] = (double *)(cold + P.c64 + (size_t)k * lp_align(8 * (size_t)m));
        active = (uint8_t *)(cold + P.active);
    }

    LPD_INLINE bool cut(int j) const { return vmask[j] != 0u; }
    LPD_INLINE bool colpresent(int c) const { return c < n || vmask[c - n] != 0u; }
    // A entry of row j at position k (variable i)
    LPD_INLINE int aent(int j, int k, int i) const
    {
        return ((vmask[j] >> k) & 1u) ? (int)sg[i] : -(int)sg[i];
    }
    LPD_INLINE double cost(int c) const { return c < n ? fabs(g[c]) : 0.0; }

    // (A v)_j for a column-space vector v (row j has a cut)
    template <typename T, typename V>
    LPD_INLINE T row_dot(int j, const V *v) const
    {
        const int e0 = cd.rowptr[j], e1 = cd.rowptr[j + 1];
        T s = (T)v[n + j];
        for (int e = e0; e < e1; ++e) {
            const int i = cd.col[e];
            const T vi = (T)v[i];
            s += aent(j, e - e0, i) > 0 ? vi : -vi;
        }
        return s;
    }
    // (A^T y)_i for standard column i, y in check space
    template <typename T, typename V>
    LPD_INLINE T col_dot(int i, const V *yy) const
    {
        T s = 0;
        for (int e = cd.colptr[i]; e < cd.colptr[i + 1]; ++e) {
            const int v = cd.vlist[e];
            const int j = v >> 5, k = v & 31;
            const uint32_t vm = vmask[j];
            if (vm) {
                const T yj = (T)yy[j];
                s += (((vm >> k) & 1u) ? (int)sg[i] : -(int)sg[i]) > 0 ? yj : -yj;
            }
        }
        return s;
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
        double s = 0.0;
        for (int k = 0; k < d; ++k) {
            const double uk = u[cd.col[e0 + k]];
            s += ((V >> k) & 1u) ? (1.0 - uk) : uk;
        }
        lhs = s;
        return s < 1.0 - o.tau_viol;
    }

    // ------------------------------------------------------------ Algorithm 7 + levels
    LPD_INLINE float wt(const float *wk, int c) const { return wk ? wk[c] : (float)d2f[c]; }

    // Column-wise greedy search for the triangular set (Algorithm 7), run as parallel rounds
    // that commit exactly the steps of the sequential algorithm with the key order
    // (weight descending, column index ascending):
    //   - a live row's candidate is the preferred degree-1 column in it (its slack always is
    //     one);
    //   - a column of residual degree rdeg >= 2 turns degree-1 once rdeg-1 of its rows are
    //     gone, i.e. when the (rdeg-1)-th largest candidate key of its rows is taken, and from
    //     then on outranks every candidate below its own key;
    //   - tau = the largest min(that key, own key) over such columns; a candidate whose key is
    //     >= tau is the sequential algorithm's choice for its row and is committed now (the
    //     best candidate overall always is, so every round makes progress).
    // Columns committed in one round never share a live row, so their updates do not race.
    // Fills pair (column of each row), pairrow (row of each chosen standard column), rnd
    // (round of each row), lf (forward-substitution level) and lb (back-substitution level).
    // Returns the number of rounds.
    LPD_INLINE int mts(const float *wk)
    {
        int *cnt = &sc->i[4];
        for (int i = tid; i < n; i += nt) {
            int dg = 0;
            for (int e = cd.colptr[i]; e < cd.colptr[i + 1]; ++e) dg += cut(cd.vlist[e] >> 5);
            status[i] = dg;
            pairrow[i] = -1;
        }
        int pl = 0;
        for (int j = tid; j < m; j += nt) {
            pair[j] = -1; rnd[j] = -1; lf[j] = -1; lb[j] = -1;
            pl += cut(j);
        }
        if (tid == 0) *cnt = 0;
        pl = block_sum1(pl, sc);
        p = pl;
        int round = 0;
        // every round commits at least one row, so pl rounds always suffice
        while (*cnt < pl && round <= pl) {
            for (int j = tid; j < m; j += nt) {
                if (!cut(j) || pair[j] >= 0) continue;
                unsigned long long best = mts_key(wt(wk, n + j), n + j);
                for (int e = cd.rowptr[j]; e < cd.rowptr[j + 1]; ++e) {
                    const int i = cd.col[e];
                    if (status[i] == 1 && pairrow[i] < 0) {
                        const unsigned long long k = mts_key(wt(wk, i), i);
                        best = k > best ? k : best;
                    }
                }
                killkey[j] = best;
            }
            if (tid == 0) sc->u64[0] = 0ull;
            __syncthreads();
            unsigned long long tau = 0ull;
            for (int i = tid; i < n; i += nt) {
                if (status[i] < 2 || pairrow[i] >= 0) continue;
                // second smallest candidate key over the live rows = (rdeg-1)-th largest
                unsigned long long k1 = ~0ull, k2 = ~0ull;
                for (int e = cd.colptr[i]; e < cd.colptr[i + 1]; ++e) {
                    const int j = cd.vlist[e] >> 5;
                    if (!cut(j) || pair[j] >= 0) continue;
                    const unsigned long long kk = killkey[j];
                    if (kk < k1) { k2 = k1; k1 = kk; }
                    else if (kk < k2) k2 = kk;
                }
                const unsigned long long own = mts_key(wt(wk, i), i);
                const unsigned long long bv = k2 < own ? k2 : own;
                tau = bv > tau ? bv : tau;
            }
            tau = wave_max(tau);
            if ((tid & 63) == 0 && tau) atomicMax(&sc->u64[0], tau);
            __syncthreads();
            tau = sc->u64[0];
            int ncom = 0;
            for (int j = tid; j < m; j += nt) {
                if (!cut(j) || pair[j] >= 0) continue;
                const unsigned long long kk = killkey[j];
                if (kk < tau) continue;
                const int c = mts_key_col(kk);
                pair[j] = c;
                rnd[j] = round;
                ++ncom;
                int L = 0;
                if (c < n) {
                    pairrow[c] = j;
                    // the other rows of c were eliminated in earlier rounds
                    for (int e = cd.colptr[c]; e < cd.colptr[c + 1]; ++e) {
                        const int jj = cd.vlist[e] >> 5;
                        if (jj != j && cut(jj)) L = max(L, lf[jj] + 1);
                    }
                }
                lf[j] = L;
                // row j is eliminated: its other waiting columns lose one degree
                for (int e = cd.rowptr[j]; e < cd.rowptr[j + 1]; ++e) {
                    const int i = cd.col[e];
                    if (i != c && pairrow[i] < 0) atomicSub(&status[i], 1);
                }
            }
            ncom = wave_sum(ncom);
            if ((tid & 63) == 0 && ncom) atomicAdd(cnt, ncom);
            __syncthreads();
            ++round;
        }
        // back-substitution levels: a row depends on the rows of the other chosen columns in
        // it, all of which were eliminated in later rounds
        for (int rd = round - 1; rd >= 0; --rd) {
            for (int j = tid; j < m; j += nt) {
                if (rnd[j] != rd) continue;
                const int c = pair[j];
                int L = 0;
                for (int e = cd.rowptr[j]; e < cd.rowptr[j + 1]; ++e) {
                    const int i = cd.col[e];
                    if (i == c) continue;
                    const int pr = pairrow[i];
                    if (pr >= 0) L = max(L, lb[pr] + 1);
                }
                lb[j] = L;
            }
            __syncthreads();
        }
        return round;
    }

    // Rows grouped by level: blist holds the rows of back-substitution level L in
    // [L ? boff[L-1] : 0, boff[L]), flist/foff likewise for forward substitution.
    LPD_INLINE void build_levels()
    {
        int mb = -1, mf = -1;
        for (int j = tid; j < m; j += nt) { mb = max(mb, lb[j]); mf = max(mf, lf[j]); }
        mb = block_max_i(mb, sc);
        mf = block_max_i(mf, sc);
        nlb = mb + 1;
        nlf = mf + 1;
        for (int k = tid; k <= m; k += nt) { boff[k] = 0; foff[k] = 0; }
        __syncthreads();
        for (int j = tid; j < m; j += nt) {
            if (lb[j] >= 0) atomicAdd(&boff[lb[j]], 1);
            if (lf[j] >= 0) atomicAdd(&foff[lf[j]], 1);
        }
        block_exscan(boff, nlb);
        block_exscan(foff, nlf);
        for (int j = tid; j < m; j += nt) {
            if (lb[j] >= 0) blist[atomicAdd(&boff[lb[j]], 1)] = j;
            if (lf[j] >= 0) flist[atomicAdd(&foff[lf[j]], 1)] = j;
        }
        __syncthreads();
    }

    // ------------------------------------------------------------ triangular solves
    // The preconditioning set M pairs every LP row j with one column pair[j]; A_M (rows by
    // paired columns) is triangular after permutation with entries +-1 (Sec. V). Vectors over
    // M's columns are stored at the row each column is paired with.
    //
    // Back-substitution out = A_M^-1 u: row j yields the value of its own column once the
    // other M-columns in row j are known (levels lb ascending).
    template <typename T, typename UF>
    LPD_INLINE void back_sub(T *out, UF u_of_row)
    {
        for (int L = 0; L < nlb; ++L) {
            const int k1 = boff[L];
            for (int k = (L ? boff[L - 1] : 0) + tid; k < k1; k += nt) {
                const int j = blist[k], c = pair[j];
                const int e0 = cd.rowptr[j], e1 = cd.rowptr[j + 1];
                T s = u_of_row(j);
                int sgn = 1;
                for (int e = e0; e < e1; ++e) {
                    const int i = cd.col[e];
                    const int a = aent(j, e - e0, i);
                    if (i == c) { sgn = a; continue; }
                    const int pr = pairrow[i];
                    if (pr >= 0) s -= a > 0 ? out[pr] : -out[pr];
                }
                out[j] = sgn > 0 ? s : -s;
            }
            __syncthreads();
        }
    }

    // Forward substitution out = A_M^-T e (out in row space): the row paired with column c
    // is solved once the other rows of c are known (levels lf ascending).
    template <typename T, typename EF>
    LPD_INLINE void fwd_sub(T *out, EF e_of_row)
    {
        for (int L = 0; L < nlf; ++L) {
            const int k1 = foff[L];
            for (int k = (L ? foff[L - 1] : 0) + tid; k < k1; k += nt) {
                const int j = flist[k], c = pair[j];
                T s = e_of_row(j);
                if (c < n) {
                    int sgn = 1;
                    for (int e = cd.colptr[c]; e < cd.colptr[c + 1]; ++e) {
                        const int v = cd.vlist[e], jj = v >> 5;
                        if (!cut(jj)) continue;
                        const int a = aent(jj, v & 31, c);
                        if (jj == j) { sgn = a; continue; }
                        s -= a > 0 ? out[jj] : -out[jj];
                    }
                    s = sgn > 0 ? s : -s;
                }
                out[j] = s;
            }
            __syncthreads();
        }
    }

    LPD_INLINE bool in_M(int c) const { return c < n ? pairrow[c] >= 0 : pair[c - n] == c; }

    // The slack columns as preconditioning set (A_M = I): used when Algorithm 7 is off.
    LPD_INLINE void slack_basis()
    {
        for (int i = tid; i < n; i += nt) pairrow[i] = -1;
        int pl = 0;
        for (int j = tid; j < m; j += nt) {
            const bool cj = cut(j);
            pair[j] = cj ? n + j : -1;
            lb[j] = cj ? 0 : -1;
            lf[j] = cj ? 0 : -1;
            pl += cj;
        }
        p = block_sum1(pl, sc);
    }

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
                if (!colpresent(c) || in_M(c)) continue;
                V.t[c] = V.dsq[c] * (c < n ? col_dot<T>(c, V.s) : V.s[c - n]);
            }
            __syncthreads();
            // f = A_M^-1 (A_N t) over s; l = h + D_M^-1 f
            T hl = 0;
            for (int L = 0; L < nlb; ++L) {
                const int k1 = boff[L];
                for (int k = (L ? boff[L - 1] : 0) + tid; k < k1; k += nt) {
                    const int j = blist[k], c = pair[j];
                    const int e0 = cd.rowptr[j], e1 = cd.rowptr[j + 1];
                    T acc = c == n + j ? (T)0 : V.t[n + j];
                    int sgn = 1;
                    for (int e = e0; e < e1; ++e) {
                        const int i = cd.col[e];
                        const int a = aent(j, e - e0, i);
                        if (i == c) { sgn = a; continue; }
                        const int pr = pairrow[i];
                        if (pr >= 0) acc -= a > 0 ? V.s[pr] : -V.s[pr];
                        else acc += a > 0 ? V.t[i] : -V.t[i];
                    }
                    const T fj = sgn > 0 ? acc : -acc;
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
            const int e0 = cd.rowptr[j], e1 = cd.rowptr[j + 1];
            double s = d2[n + j] * dy[j];
            for (int e = e0; e < e1; ++e) {
                const int i = cd.col[e];
                s += aent(j, e - e0, i) > 0 ? tq[i] : -tq[i];
            }
            const double rj = w[j] - s;
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
        CG<PT> V1 = {r, yv, h, l, zz, t, idm, om, d2f};
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
                // undo the round: its correction is the forward substitution left in f64 only
                // when mu = 0, so recompute it from the stored dy difference
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
        double v = dd < 1e-30 ? 1e-30 : (dd > 1e30 ? 1e30 : dd);
        d2f[c] = (PT)v;
    }

    // ------------------------------------------------------------ interior-point method
    // Infeasible primal-dual path-following method of Sec. IV-B on the LP of the current
    // cut set (rows = checks with a cut): residuals r_b = b - Ax, r_c = c - A^T y - z,
    // mu = sigma x^T z / q, r_e = mu e - XZe, D^2 = X Z^-1; Newton direction from
    // (A D^2 A^T) dy = r_b + A D^2 r_c - A Z^-1 r_e, dx = D^2 A^T dy - D^2 r_c + Z^-1 r_e,
    // dz = X^-1 (r_e - Z dx); separate primal and dual step lengths (fraction eta of the
    // distance to the boundary, at most 1). Starts at x = e, y = 0, z = e; stops when
    // x^T z / (1 + |c^T x|), ||r_b|| / (1 + ||b||) and ||r_c|| / (1 + ||c||) are all < eps.
    // Returns 0 or a negative LPDEC_FLAG_*.
    LPD_INLINE int ipm(lpdec_stats &st, int &iters)
    {
        double a0[2] = {0.0, 0.0};
        for (int j = tid; j < m; j += nt) {
            if (cut(j)) {
                // b of the flipped parity inequality: |V| - 1 - sum of its u-coefficients
                // over variables with sigma_i = -1
                const uint32_t V = vmask[j];
                const int e0 = cd.rowptr[j], e1 = cd.rowptr[j + 1];
                int vsz = 0, sneg = 0;
                for (int e = e0; e < e1; ++e) {
                    const int s = ((V >> (e - e0)) & 1u) ? 1 : -1;
                    vsz += s > 0;
                    if (sg[cd.col[e]] < 0) sneg += s;
                }
                const double bj = (double)(vsz - 1 - sneg);
                b[j] = bj;
                a0[0] += bj * bj;
                x[n + j] = 1.0; z[n + j] = 1.0;
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
            if (o.precond) st.mts_rounds += mts(nullptr);
            else slack_basis();
            build_levels();
            st.max_levels = max(st.max_levels, max(nlb, nlf));
            const long long t1 = wall_clock64();
            double resid2;
            const int pits = solve(mu, st.ref_rounds, st.escalations, resid2);
            const long long t2 = wall_clock64();
            st.ticks_mts += t1 - t0;
            st.ticks_solve += t2 - t1;
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
            int its = 0;
            int pl = 0;
            for (int j = tid; j < m; j += nt) pl += cut(j);
            p = block_sum1(pl, sc);
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
            status_xh(i, xh);
            a.xhat[(size_t)f * n + i] = (uint8_t)xh;
            if (a.u_out) a.u_out[(size_t)f * n + i] = ui;
        }
        fr = block_max_d(fr, sc);
        ob = block_sum1(ob, sc);
        int syn = 0;
        for (int j = tid; j < m; j += nt) {
            int par = 0;
            for (int e = cd.rowptr[j]; e < cd.rowptr[j + 1]; ++e) par ^= this->status[cd.col[e]];
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

    // the decision bits are kept in the residual-degree array for the syndrome
    LPD_INLINE void status_xh(int i, int v) { this->status[i] = v; }
};

}  // namespace lpdec
