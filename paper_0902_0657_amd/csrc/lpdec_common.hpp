// Shared host/device definitions of the decoder: options, code view, per-frame memory plan.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "../../include/lpdec.h"

namespace lpdec {

// Options as the kernels see them.
struct Opts {
    int malp_mode;   // 0: MALP-A, 1: MALP-B
    int malp_max;
    int ipm_max;
    int pcg_maxit;
    int ref_max;
    int precond;     // 1: triangular preconditioner, 0: M = I
    int direct;      // 1: dense Cholesky fallback for Newton solves PCG does not finish
    int mts_reuse;   // the triangular set is searched on every mts_reuse-th IPM iteration of an LP
    int warm;        // 1: a Newton solve starts from the previous direction of the same LP
    double ipm_warm; // > 0: an LP after the first starts from the previous LP's point, shifted by this
    double tau_viol, tau_act, tau_int;
    double eps, eps_stall, sigma, eta;
    double tau_cost; // a cost decrease between successive LPs beyond tau_cost (1 + c^T x) fails the decode
    double pcg_tol, ref_tol, xi_tol;
};

// Device view of one parity-check matrix H (rows = checks, columns = variables).
struct CodeView {
    int m, n, E;
    int dcmax, dvmax;    // largest check / variable degree
    const int *rowptr;   // [m+1] CSR
    const int *col;      // [E]   variable of each CSR edge (ascending within a row)
    const int *colptr;   // [n+1] CSC
    const int *vlist;    // [E]   CSC entries: (check << 5) | position of the variable in the check's row
};

// Byte offsets of every per-frame array. "hot" arrays are touched by every PCG iteration or
// by the triangular-set search; they live in LDS when they fit (else in the frame's global
// workspace). "cold" arrays hold the FP64 interior-point state in the global workspace.
// Index lists are uint16 (bit 15 = negative coefficient, bit 14 = row reference, bits
// 0..13 = index), which bounds n + m by 16383. Row-type lists (rlist, bins) use slots of rw
// entries (a multiple of 8: one 16-byte load per 8), column-type lists (clist, fins) slots
// of cw entries (a multiple of 4: one 8-byte load per 4), padded with the end marker.
struct Plan {
    int rw, cw;                                // slot widths (entries)
    int lanecols, maskwords;                   // columns per lane of Algorithm 7, mask words
    int dense_on;                              // the dense fallback region exists
    // hot
    size_t h, r, v, l, idm, om, st, d2f;       // PT: [m] x 6, st [m + (n+m) + 1], d2f [n+m]
    size_t rlist, clist, bins, fins;           // u16 [m*rw], [n*cw], [m*rw], [m*cw]
    size_t pair, pairrow, lbv, lfv, order;     // i16 [m], [n], [m], [m], [m]
    size_t boff, foff;                         // i32 [m+1]
    size_t deg, sg;                            // u8 / i8 [n]
    size_t rdeg, r1;                           // Algorithm 8: u8 [m] row degrees, u32 [(m+31)/32] degree-1 rows
    size_t vmask;                              // u32 [m]
    size_t rank, lcol, lmask;                  // u8 [n+m], u16 [64*lanecols], u32 [64*maskwords]
    size_t hot_bytes;
    // cold, FP64 unless noted
    size_t x, z, dx, dz, rc, tq, d2;           // [n+m]
    size_t y, dy, rb, w, b, rho, f64;          // [m]
    size_t c64;                                // 8 x [m]: FP64 PCG vectors (escalation), dy copy
    size_t st64;                               // [m + (n+m) + 1]: s | t of the escalated PCG
    size_t ridx, colk, dense;                  // dense fallback: i32 [m+1], FP64 [mp], FP64 [mp*mp], mp = m rounded up to kDenseTile
    size_t u, g;                               // [n]
    size_t active;                             // u8 [m]
    size_t vprev;                              // u32 [m]: cut of each check in the previous LP
    size_t vback;                              // u32 [m]: cut of each check two LPs back
    size_t cold_bytes;
};

__host__ __device__ inline size_t lp_align(size_t v) { return (v + 15) & ~(size_t)15; }

// LDS of the dense fallback: the factor of the current diagonal tile (32 x 32 FP64), the
// reciprocals of its diagonal and one block of the substitution vector
constexpr int kDenseTile = 32;
constexpr size_t kDenseLdsBytes = (kDenseTile * kDenseTile + 2 * kDenseTile) * 8;

__host__ __device__ inline int lp_pow2_at_least(int v, int lo)
{
    int w = lo;
    while (w < v) w <<= 1;
    return w;
}

__host__ __device__ inline Plan make_plan(int m, int n, int dc, int dv, int pt_size, bool dense = false)
{
    Plan p;
    // a row slot holds a header and up to dc entries (row lists: dc columns), a column slot
    // a header and up to dv - 1 entries (column lists: dv rows)
    p.rw = lp_pow2_at_least(dc + 1, 8);
    p.cw = lp_pow2_at_least(dv, 4);
    p.lanecols = (n + m + 63) / 64;
    p.maskwords = (p.lanecols + 31) / 32;
    size_t o = 0;
    const size_t M = (size_t)m, N = (size_t)n, Q = (size_t)n + m, P = (size_t)pt_size;
    const size_t DC = (size_t)p.rw, DV = (size_t)p.cw;
    p.h = o; o = lp_align(o + P * M);
    p.r = o; o = lp_align(o + P * M);
    p.v = o; o = lp_align(o + P * M);
    p.l = o; o = lp_align(o + P * M);
    p.idm = o; o = lp_align(o + P * M);
    p.om = o; o = lp_align(o + P * M);
    p.st = o; o = lp_align(o + P * (M + Q + 1));
    p.d2f = o; o = lp_align(o + P * Q);
    p.vmask = o; o = lp_align(o + 4 * M);
    p.boff = o; o = lp_align(o + 4 * (M + 1));
    p.foff = o; o = lp_align(o + 4 * (M + 1));
    p.lmask = o; o = lp_align(o + 4 * 64 * (size_t)p.maskwords);
    p.rlist = o; o = lp_align(o + 2 * M * DC);
    p.clist = o; o = lp_align(o + 2 * N * DV);
    p.bins = o; o = lp_align(o + 2 * M * DC);
    p.fins = o; o = lp_align(o + 2 * M * DV);
    p.lcol = o; o = lp_align(o + 2 * 64 * (size_t)p.lanecols);
    p.rank = o; o = lp_align(o + Q);
    p.pair = o; o = lp_align(o + 2 * M);
    p.pairrow = o; o = lp_align(o + 2 * N);
    p.lbv = o; o = lp_align(o + 2 * M);
    p.lfv = o; o = lp_align(o + 2 * M);
    p.order = o; o = lp_align(o + 2 * M);
    p.deg = o; o = lp_align(o + N);
    p.sg = o; o = lp_align(o + N);
    p.rdeg = o; o = lp_align(o + M);
    p.r1 = o; o = lp_align(o + 4 * ((M + 31) / 32));
    p.hot_bytes = o;
    o = 0;
    p.x = o; o = lp_align(o + 8 * Q);
    p.z = o; o = lp_align(o + 8 * Q);
    p.dx = o; o = lp_align(o + 8 * Q);
    p.dz = o; o = lp_align(o + 8 * Q);
    p.rc = o; o = lp_align(o + 8 * Q);
    p.tq = o; o = lp_align(o + 8 * Q);
    p.d2 = o; o = lp_align(o + 8 * Q);
    p.y = o; o = lp_align(o + 8 * M);
    p.dy = o; o = lp_align(o + 8 * M);
    p.rb = o; o = lp_align(o + 8 * M);
    p.w = o; o = lp_align(o + 8 * M);
    p.b = o; o = lp_align(o + 8 * M);
    p.rho = o; o = lp_align(o + 8 * M);
    p.f64 = o; o = lp_align(o + 8 * M);
    p.c64 = o; o = o + 8 * lp_align(8 * M);
    p.st64 = o; o = lp_align(o + 8 * (M + Q + 1));
    p.dense_on = dense ? 1 : 0;
    p.ridx = o; o = lp_align(o + 4 * (M + 1));
    // the dense system is padded to a whole number of kDenseTile rows
    const size_t MP = (M + kDenseTile - 1) / kDenseTile * kDenseTile;
    p.colk = o; o = lp_align(o + 8 * MP);
    p.dense = o; o = lp_align(o + (dense ? 8 * MP * MP : 0));
    p.u = o; o = lp_align(o + 8 * N);
    p.g = o; o = lp_align(o + 8 * N);
    p.active = o; o = lp_align(o + M);
    p.vprev = o; o = lp_align(o + 4 * M);
    p.vback = o; o = lp_align(o + 4 * M);
    p.cold_bytes = o;
    return p;
}

// What a launch asks the decode kernel to do.
enum Mode : int {
    MODE_DECODE = 0,      // full MALP decode
    MODE_IPM = 1,         // one LP (cut set given) -> x, y, z
    MODE_SOLVE = 2,       // one Newton solve on given d2, w
    MODE_MATVEC = 3,      // l = A D^2 A^T h
    MODE_MTS = 4,         // Algorithm 7 + levels
    MODE_CUTS = 5,        // Algorithm 2 on every check
    MODE_SERVE = 6,       // persistent: frames claimed from a host ring until idle or stopped
};

// Kernel arguments (one struct, passed by value).
struct Args {
    CodeView code;
    const CodeView *codes;     // MODE_IPM, nullable: [nframes] a matrix per frame (same m and n)
    Opts o;
    Plan plan;
    int nframes;
    int mode;
    int hot_in_lds;
    char *hot_ws;          // per-frame hot arena in global memory when not in LDS
    char *cold_ws;         // per-frame cold arena
    size_t hot_stride, cold_stride;
    // inputs
    const void *gamma;     // [nframes*n] float or double
    int gamma_f64;
    const uint32_t *vmask_in;  // [nframes*m]   (IPM, SOLVE, MATVEC)
    const uint8_t *hascut_in;  // [nframes*m]   (MTS)
    const float *w_in;         // [nframes*(n+m)] (MTS)
    const double *d2_in;       // [nframes*(n+m)] (SOLVE, MATVEC)
    const double *vec_in;      // [nframes*m] h (MATVEC) or w (SOLVE); [nframes*n] u (CUTS)
    // outputs
    uint8_t *xhat;             // [nframes*n]
    int32_t *flag;             // [nframes]
    double *obj;               // [nframes]
    int32_t *done;             // [nframes], nullable: set to 1 once the frame's outputs are
                               // visible to the host (outputs in host-mapped memory)
    const int32_t *order;      // MODE_DECODE with next, nullable: the k-th frame taken is order[k]
    int32_t *next;             // MODE_DECODE, nullable: a grid smaller than the batch, whose
                               // workgroups take frames in turn from *next (zero at launch)
    // MODE_SERVE: frames are ring slots; ticket t (claimed once, in order, from claim[0] while
    // t < *published) is slot t mod ring. claim[1] counts the workgroups holding or claiming a
    // ticket; claim[2] closes the launch: set by a workgroup that has polled idle_polls times
    // in a row (about 54 us apart) while no ticket was held or unclaimed, it makes every
    // workgroup leave. A workgroup also leaves when *stop is set or its index is not below
    // *share
    int32_t *claim;            // device memory, claim[1] and claim[2] zero at launch
    const int32_t *published;  // host-mapped
    const int32_t *stop;       // host-mapped
    const int32_t *share;      // host-mapped
    int ring;
    int idle_polls;
    lpdec_stats *stats;        // [nframes]
    double *u_out;             // [nframes*n]
    uint32_t *trace;           // [nframes*trace_cap*m]
    int trace_cap;
    double *vec_out;           // y (SOLVE) [nframes*m], l (MATVEC) [nframes*m], lhs (CUTS)
    double *x_out, *z_out;     // [nframes*(n+m)] (IPM)
    int32_t *i_out;            // iterations / pair / rounds
    int32_t *i_out2, *i_out3;  // status / lev_b / lev_f
    double *d_out;             // residual (SOLVE)
    uint32_t *u32_out;         // vmask (CUTS)
    uint8_t *u8_out;           // viol (CUTS)
};

}  // namespace lpdec
