/*
 * lpdec_oracle.c -- plain FP64 CPU oracle for adaptive LP decoding.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library. The GPU library shares no code with it.
 *
 * What it computes (Taghavi, Shokrollahi, Siegel, "Efficient Implementation of Linear
 * Programming Decoding"):
 *   - Algorithm 2: the violated parity inequality of one check, if any (Sec. III).
 *   - Algorithm 3 (MALP-A) and its variant MALP-B (Sec. III-A), at most one cut per check
 *     (Theorem 3), over the LP in the standard matrix form of Sec. III-A converted to the
 *     augmented form of Sec. IV-B (variable flip x_i = u_i or 1-u_i, one slack per cut).
 *   - The infeasible primal-dual path-following interior-point method of Sec. IV-B:
 *     residuals r_b, r_c, r_e, the reduced Newton equations for dy, dx, dz, separate primal
 *     and dual step lengths, mu proportional to the duality gap.
 *     The normal equations (A D^2 A^T) dy = w are solved by a direct Cholesky factorisation
 *     (the standard direct method named in Sec. IV-C), NOT by PCG.
 *   - Algorithm 7 (column-wise greedy search for the maximum-weight triangular set), with
 *     the binary heap of Sec. V-B, and the dependency levels of the two triangular solves.
 *   - Algorithm 8 (row-wise greedy search) with the diagonal or the triangular expansion of
 *     Sec. V-B, and the levels of any triangular set.
 *   - Algorithm 6 (incremental greedy search) with the Triangulation Step of Algorithm 5.
 *   - ALP decoding (Algorithm 1): all cuts kept, several per check possible.
 *   - Algorithm 4 (PCG) in FP64 with the preconditioner M = A_M D_M^2 A_M^T of Sec. V,
 *     used only as a reference in tests (the decoder itself uses Cholesky).
 *
 * Readings where the paper is silent (all documented in the design notes):
 *   mu = sigma_c * x^T z / q with sigma_c = 0.1; fraction-to-boundary steps with eta = 0.9995;
 *   start x = e, y = 0, z = e; stop when x^T z/(1+|c^T x|), ||r_b||/(1+||b||) and
 *   ||r_c||/(1+||c||) are all below eps (1e-8), or, once the largest of the three is below
 *   eps_stall (1e-7), when it has not at least halved over the last two iterations (the
 *   numerical floor of a degenerate LP in double precision); a cut is violated when its left-hand side is
 *   below 1 - tau_viol; a cut is inactive when its slack exceeds max(tau_act, its dual slack);
 *   u_i > 1/2 strict in Algorithm 2 and argmin ties go to the lowest variable index;
 *   Algorithm 7 orders columns by (float(d_i^2) descending, column index ascending), slack
 *   columns numbered after the n standard columns in ascending check order; Algorithm 8
 *   takes the lowest-indexed degree-1 row and removes the column of smallest
 *   (float(d_i^2), index).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int malp_mode;   /* 0: MALP-A, 1: MALP-B */
    int malp_max;    /* cap on MALP iterations (LPs solved) */
    int ipm_max;     /* cap on IPM iterations per LP */
    double tau_viol; /* violation threshold of Algorithm 2 */
    double tau_act;  /* active-cut threshold */
    double tau_int;  /* integrality threshold of the output */
    double sigma_c;  /* centering factor of mu */
    double eta;      /* fraction-to-boundary factor */
    double eps;      /* IPM termination tolerance */
    double eps_stall;/* below it, an iteration that makes no progress ends the IPM */
    double tau_cost; /* a cost decrease beyond tau_cost (1 + |c^T x|) between LPs is a failure */
    int box_clamp;   /* 1: u^k is put back on [0, 1]^n before Algorithm 2 (tests set 0) */
    int cycle_stop;  /* 1: a cut set that recurs two LPs later ends the decode (tests set 0) */
} orc_opts;

typedef struct {
    int malp_iters;      /* LPs solved */
    int ipm_iters;       /* IPM iterations summed over LPs */
    int p_max;           /* largest number of cuts in one LP */
    int p_final;         /* cuts in the last LP */
    int status;          /* 0 ok, -1 IPM cap, -3 MALP cap, -2 non-finite, -5 cost decrease,
                            -7 cut cycle */
} orc_stats;

/* ------------------------------------------------------------------------------------ */
/* Algorithm 2: the (at most one, Theorem 1) violated parity inequality of a check.       */
/* u[k] is the value of the k-th neighbour (neighbours in ascending variable order).      */
/* V is returned as a bit mask over neighbour positions. Returns 1 when violated.         */
int orc_find_cut(int d, const double *u, double tau_viol, uint32_t *vmask, double *lhs_out)
{
    uint32_t S = 0;
    int cnt = 0;
    for (int k = 0; k < d; ++k)
        if (u[k] > 0.5) { S |= 1u << k; ++cnt; }
    uint32_t V = S;
    if ((cnt & 1) == 0) {
        /* |S| even: flip membership of the entry closest to 1/2 */
        int ks = 0;
        double best = fabs(u[0] - 0.5);
        for (int k = 1; k < d; ++k) {
            double a = fabs(u[k] - 0.5);
            if (a < best) { best = a; ks = k; }
        }
        V = S ^ (1u << ks);
    }
    /* left-hand side of the parity inequality in its ">= 1" form */
    double lhs = 0.0;
    for (int k = 0; k < d; ++k)
        lhs += ((V >> k) & 1u) ? (1.0 - u[k]) : u[k];
    *vmask = V;
    *lhs_out = lhs;
    return lhs < 1.0 - tau_viol;
}

/* ------------------------------------------------------------------------------------ */
/* The LP of one MALP iteration in augmented form: min c^T x, A x = b, x >= 0.            */
/* Rows = checks that carry a cut, in ascending check order. Columns 0..n-1 are the       */
/* flipped standard variables, column n+r is the slack of row r.                           */
typedef struct {
    int n, p, q;
    int *rowchk;           /* [p] check of row r */
    int *rptr, *ridx;      /* CSR of the standard block (entries +-1) */
    signed char *rval;
    int *cptr, *cidx;      /* CSC of the standard block */
    signed char *cval;
    double *b, *c;         /* [p], [q] */
} lp_t;

static void lp_free(lp_t *lp)
{
    free(lp->rowchk); free(lp->rptr); free(lp->ridx); free(lp->rval);
    free(lp->cptr); free(lp->cidx); free(lp->cval); free(lp->b); free(lp->c);
    memset(lp, 0, sizeof(*lp));
}

/* The LP of a list of cuts: cut r comes from check chk[r] with odd set V[r] (bit k = k-th
   neighbour of the check). sigma_i = +1 when gamma_i >= 0 (the box constraint u_i >= 0 is
   kept), else -1. MALP's LPs list at most one cut per check, in ascending check order; ALP's
   can hold several cuts of one check. */
static void lp_build_cuts(lp_t *lp, int n, const int *rowptr, const int *col, const double *gamma,
                          int p, const int *chk, const uint32_t *Vs)
{
    int nnz = 0;
    for (int r = 0; r < p; ++r) nnz += rowptr[chk[r] + 1] - rowptr[chk[r]];
    lp->n = n; lp->p = p; lp->q = n + p;
    lp->rowchk = malloc(sizeof(int) * (p + 1));
    lp->rptr = malloc(sizeof(int) * (p + 1));
    lp->ridx = malloc(sizeof(int) * (nnz + 1));
    lp->rval = malloc(nnz + 1);
    lp->b = malloc(sizeof(double) * (p + 1));
    lp->c = malloc(sizeof(double) * (n + p + 1));
    int e = 0;
    lp->rptr[0] = 0;
    for (int r = 0; r < p; ++r) {
        const int j = chk[r];
        uint32_t V = Vs[r];
        int vsz = 0;
        int sneg = 0;
        for (int t = rowptr[j]; t < rowptr[j + 1]; ++t) {
            int k = t - rowptr[j];
            int i = col[t];
            int sv = ((V >> k) & 1u) ? 1 : -1;     /* coefficient of u_i in A u <= b */
            int sig = gamma[i] >= 0.0 ? 1 : -1;
            if ((V >> k) & 1u) ++vsz;
            if (sig < 0) sneg += sv;                 /* u_i = 1 - x_i moves sv to the rhs */
            lp->ridx[e] = i;
            lp->rval[e] = (signed char)(sig * sv);
            ++e;
        }
        lp->rowchk[r] = j;
        lp->b[r] = (double)(vsz - 1) - (double)sneg;
        lp->rptr[r + 1] = e;
    }
    for (int i = 0; i < n; ++i) lp->c[i] = fabs(gamma[i]);
    for (int k = 0; k < p; ++k) lp->c[n + k] = 0.0;
    /* column view of the standard block */
    lp->cptr = calloc(n + 1, sizeof(int));
    lp->cidx = malloc(sizeof(int) * (nnz + 1));
    lp->cval = malloc(nnz + 1);
    for (int t = 0; t < nnz; ++t) lp->cptr[lp->ridx[t] + 1]++;
    for (int i = 0; i < n; ++i) lp->cptr[i + 1] += lp->cptr[i];
    int *fill = malloc(sizeof(int) * (n + 1));
    memcpy(fill, lp->cptr, sizeof(int) * n);
    for (int rr = 0; rr < p; ++rr)
        for (int t = lp->rptr[rr]; t < lp->rptr[rr + 1]; ++t) {
            int i = lp->ridx[t];
            lp->cidx[fill[i]] = rr;
            lp->cval[fill[i]] = lp->rval[t];
            fill[i]++;
        }
    free(fill);
}

/* The LP of a cut set with at most one cut per check: mask[j] = V of check j's cut, 0 = none. */
static void lp_build(lp_t *lp, int m, int n, const int *rowptr, const int *col,
                     const double *gamma, const uint32_t *mask)
{
    int p = 0;
    for (int j = 0; j < m; ++j) p += mask[j] != 0;
    int *chk = malloc(sizeof(int) * (p + 1));
    uint32_t *Vs = malloc(sizeof(uint32_t) * (p + 1));
    p = 0;
    for (int j = 0; j < m; ++j)
        if (mask[j]) { chk[p] = j; Vs[p] = mask[j]; ++p; }
    lp_build_cuts(lp, n, rowptr, col, gamma, p, chk, Vs);
    free(chk); free(Vs);
}

/* y = A x  (length p) */
static void lp_Ax(const lp_t *lp, const double *x, double *y)
{
    for (int r = 0; r < lp->p; ++r) {
        double s = x[lp->n + r];
        for (int t = lp->rptr[r]; t < lp->rptr[r + 1]; ++t) s += lp->rval[t] * x[lp->ridx[t]];
        y[r] = s;
    }
}

/* x = A^T y  (length q) */
static void lp_ATy(const lp_t *lp, const double *y, double *x)
{
    for (int i = 0; i < lp->n; ++i) {
        double s = 0.0;
        for (int t = lp->cptr[i]; t < lp->cptr[i + 1]; ++t) s += lp->cval[t] * y[lp->cidx[t]];
        x[i] = s;
    }
    for (int r = 0; r < lp->p; ++r) x[lp->n + r] = y[r];
}

static double dot(const double *a, const double *b, int k)
{
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += a[i] * b[i];
    return s;
}

/* Dense Cholesky of the p x p normal matrix Q = A D^2 A^T, assembled column by column.
   A pivot that is not safely positive is replaced by a huge value (standard IPM practice),
   which sets the matching component of the solution to about zero. */
static void normal_matrix(const lp_t *lp, const double *d2, double *Q)
{
    int p = lp->p;
    memset(Q, 0, sizeof(double) * (size_t)p * p);
    for (int i = 0; i < lp->n; ++i)
        for (int s = lp->cptr[i]; s < lp->cptr[i + 1]; ++s)
            for (int t = lp->cptr[i]; t < lp->cptr[i + 1]; ++t)
                Q[(size_t)lp->cidx[s] * p + lp->cidx[t]] += d2[i] * lp->cval[s] * lp->cval[t];
    for (int r = 0; r < p; ++r) Q[(size_t)r * p + r] += d2[lp->n + r];
}

static void cholesky(double *Q, int p)
{
    double dmax = 0.0;
    for (int r = 0; r < p; ++r) if (Q[(size_t)r * p + r] > dmax) dmax = Q[(size_t)r * p + r];
    for (int k = 0; k < p; ++k) {
        double *Lk = Q + (size_t)k * p;
        double s = Lk[k];
        for (int t = 0; t < k; ++t) s -= Lk[t] * Lk[t];
        if (!(s > 1e-30 * dmax)) s = 1e128;
        double lkk = sqrt(s);
        Lk[k] = lkk;
        for (int i = k + 1; i < p; ++i) {
            double *Li = Q + (size_t)i * p;
            double v = Li[k];
            for (int t = 0; t < k; ++t) v -= Li[t] * Lk[t];
            Li[k] = v / lkk;
        }
    }
}

static void chol_solve(const double *L, int p, const double *w, double *x)
{
    for (int i = 0; i < p; ++i) {
        double s = w[i];
        for (int t = 0; t < i; ++t) s -= L[(size_t)i * p + t] * x[t];
        x[i] = s / L[(size_t)i * p + i];
    }
    for (int i = p - 1; i >= 0; --i) {
        double s = x[i];
        for (int t = i + 1; t < p; ++t) s -= L[(size_t)t * p + i] * x[t];
        x[i] = s / L[(size_t)i * p + i];
    }
}

/* One Newton direction of the infeasible primal-dual method (Sec. IV-B):
     (A D^2 A^T) dy = r_b + A D^2 r_c - A Z^-1 r_e
     dx = D^2 A^T dy - D^2 r_c + Z^-1 r_e
     dz = X^-1 (r_e - Z dx)
   with r_b = b - A x, r_c = c - A^T y - z, r_e = mu e - X Z e, D^2 = X Z^-1.
   Work arrays: Q [p*p], t1 [q], t2 [q]. */
static void newton(const lp_t *lp, const double *x, const double *y, const double *z, double mu,
                   double *dx, double *dy, double *dz, double *rb, double *rc,
                   double *Q, double *t1, double *t2)
{
    int p = lp->p, q = lp->q;
    lp_Ax(lp, x, rb);
    for (int r = 0; r < p; ++r) rb[r] = lp->b[r] - rb[r];
    lp_ATy(lp, y, rc);
    for (int i = 0; i < q; ++i) rc[i] = lp->c[i] - rc[i] - z[i];
    double *d2 = t2;
    for (int i = 0; i < q; ++i) d2[i] = x[i] / z[i];
    /* t1 = D^2 r_c - Z^-1 r_e */
    for (int i = 0; i < q; ++i) t1[i] = d2[i] * rc[i] - (mu - x[i] * z[i]) / z[i];
    double *w = dz;  /* borrow dz (length q >= p) for the right-hand side */
    lp_Ax(lp, t1, w);
    for (int r = 0; r < p; ++r) w[r] += rb[r];
    normal_matrix(lp, d2, Q);
    cholesky(Q, p);
    chol_solve(Q, p, w, dy);
    lp_ATy(lp, dy, t1);
    for (int i = 0; i < q; ++i) {
        double re = mu - x[i] * z[i];
        dx[i] = d2[i] * t1[i] - d2[i] * rc[i] + re / z[i];
    }
    for (int i = 0; i < q; ++i) {
        double re = mu - x[i] * z[i];
        dz[i] = (re - z[i] * dx[i]) / x[i];
    }
}

static double norm2(const double *a, int k) { return sqrt(dot(a, a, k)); }

/* Infeasible primal-dual path-following IPM on one LP. Returns 0 when converged,
   -1 at the iteration cap, -2 on a non-finite iterate. */
static int ipm_solve(const lp_t *lp, const orc_opts *o, double *x, double *y, double *z, int *iters)
{
    int p = lp->p, q = lp->q;
    for (int i = 0; i < q; ++i) { x[i] = 1.0; z[i] = 1.0; }
    for (int r = 0; r < p; ++r) y[r] = 0.0;
    double *dx = malloc(sizeof(double) * q), *dz = malloc(sizeof(double) * q);
    double *dy = malloc(sizeof(double) * (p + 1)), *rb = malloc(sizeof(double) * (p + 1));
    double *rc = malloc(sizeof(double) * q), *t1 = malloc(sizeof(double) * q);
    double *t2 = malloc(sizeof(double) * q);
    double *Q = malloc(sizeof(double) * ((size_t)p * p + 1));
    double nb = norm2(lp->b, p), nc = norm2(lp->c, q);
    int it, status = -1;
    double phi1 = INFINITY, phi2 = INFINITY;   /* error measure one and two iterations ago */
    for (it = 0; it < o->ipm_max; ++it) {
        lp_Ax(lp, x, rb);
        for (int r = 0; r < p; ++r) rb[r] = lp->b[r] - rb[r];
        lp_ATy(lp, y, rc);
        for (int i = 0; i < q; ++i) rc[i] = lp->c[i] - rc[i] - z[i];
        double gap = dot(x, z, q);
        double cx = dot(lp->c, x, q);
        if (!isfinite(gap) || !isfinite(cx)) { status = -2; break; }
        double e1 = gap / (1.0 + fabs(cx)), e2 = norm2(rb, p) / (1.0 + nb);
        double e3 = norm2(rc, q) / (1.0 + nc);
        double phi = fmax(e1, fmax(e2, e3));
        if (phi < o->eps) { status = 0; break; }
        /* stalled at the floor of double precision: accept the iterate */
        if (phi < o->eps_stall && phi > 0.5 * phi2) { status = 0; break; }
        phi2 = phi1;
        phi1 = phi;
        double mu = o->sigma_c * gap / q;
        newton(lp, x, y, z, mu, dx, dy, dz, rb, rc, Q, t1, t2);
        double bp = 1.0, bd = 1.0;
        for (int i = 0; i < q; ++i) {
            if (dx[i] < 0.0) { double s = -x[i] / dx[i]; if (o->eta * s < bp) bp = o->eta * s; }
            if (dz[i] < 0.0) { double s = -z[i] / dz[i]; if (o->eta * s < bd) bd = o->eta * s; }
        }
        for (int i = 0; i < q; ++i) { x[i] += bp * dx[i]; z[i] += bd * dz[i]; }
        for (int r = 0; r < p; ++r) y[r] += bd * dy[r];
    }
    *iters = it;
    free(dx); free(dz); free(dy); free(rb); free(rc); free(t1); free(t2); free(Q);
    return status;
}

/* ------------------------------------------------------------------------------------ */
/* MALP-A / MALP-B decoding (Algorithm 3 and its variant B).                               */
int orc_decode(int m, int n, const int *rowptr, const int *col, const double *gamma,
               const orc_opts *o, double *u_out, uint8_t *xhat, int *flag, double *obj,
               orc_stats *st, uint32_t *trace_mask, double *trace_obj, int *trace_p,
               int *trace_ipm, int trace_cap)
{
    uint32_t *mask = calloc(m, sizeof(uint32_t));     /* V of the cut of each check, 0 = none */
    uint8_t *active = calloc(m, 1);
    double *u = malloc(sizeof(double) * n);
    double *nb = malloc(sizeof(double) * 64);
    double *x = malloc(sizeof(double) * (n + m)), *z = malloc(sizeof(double) * (n + m));
    double *y = malloc(sizeof(double) * (m + 1));
    orc_stats s = {0, 0, 0, 0, 0};
    /* initial LP: box constraints only; its solution is the bit-wise hard decision */
    double gneg = 0.0;                                /* gamma^T u at the hard decision */
    for (int i = 0; i < n; ++i) {
        u[i] = gamma[i] >= 0.0 ? 0.0 : 1.0;
        if (gamma[i] < 0.0) gneg += gamma[i];
    }
    double cost_prev = gneg;                          /* gamma^T u^(k-1) */
    double cost_prev2 = gneg;                         /* gamma^T u^(k-2) */
    uint32_t *mask1 = calloc(m, sizeof(uint32_t));    /* cut set of LP k-1 */
    uint32_t *mask2 = calloc(m, sizeof(uint32_t));    /* cut set of LP k-2 */
    int last = 0;                                     /* the LP about to be solved is the last */
    int k;
    for (k = 0; k < o->malp_max; ++k) {
        int added = 0;
        if (o->malp_mode == 1)
            for (int j = 0; j < m; ++j) if (mask[j] && !active[j]) mask[j] = 0;
        for (int j = 0; j < m; ++j) {
            if (mask[j] && active[j]) continue;   /* a check with an active cut is skipped */
            int d = rowptr[j + 1] - rowptr[j];
            for (int t = 0; t < d; ++t) nb[t] = u[col[rowptr[j] + t]];
            uint32_t V;
            double lhs;
            if (orc_find_cut(d, nb, o->tau_viol, &V, &lhs)) {
                mask[j] = V;                      /* replaces the check's inactive cut, if any */
                active[j] = 0;
                added = 1;
            }
        }
        if (!added) break;
        /* Theorem 2b rules out a recurring cut set: LP k equal to LP k-2 can only come from
           an optimum that is not unique at the IPM's accuracy (the uniqueness the theorem
           assumes), where a cut that bounds the optimum looks inactive. The steps are
           deterministic, so the two LPs would then alternate until the cap. The decode ends
           with the solution of the costlier of the two: u^(k-1) as it stands, or LP k (the
           same LP as LP k-2) solved once more. */
        if (o->cycle_stop && k >= 2 && !memcmp(mask, mask2, sizeof(uint32_t) * m)) {
            s.status = -7;
            if (cost_prev >= cost_prev2) break;
            last = 1;
        }
        memcpy(mask2, mask1, sizeof(uint32_t) * m);
        memcpy(mask1, mask, sizeof(uint32_t) * m);
        lp_t lp;
        lp_build(&lp, m, n, rowptr, col, gamma, mask);
        int its = 0;
        int rc = ipm_solve(&lp, o, x, y, z, &its);
        s.malp_iters++;
        s.ipm_iters += its;
        if (lp.p > s.p_max) s.p_max = lp.p;
        s.p_final = lp.p;
        /* u^k from the LP solution (Sec. IV-B variable flip). Every u^k satisfies the box
           constraints (Theorem 2a), which are not all in the LP: a coordinate the IPM leaves
           slightly outside [0, 1] (one whose cost |gamma_i| is too small for the gap test to
           pin it) is put back on the box before Algorithm 2 looks at it, so that rounding
           cannot produce a violated cut (Theorem 1 assumes u in [0, 1]^n). */
        double cost = 0.0;
        for (int i = 0; i < n; ++i) {
            double ui = gamma[i] >= 0.0 ? x[i] : 1.0 - x[i];
            if (o->box_clamp) ui = ui < 0.0 ? 0.0 : (ui > 1.0 ? 1.0 : ui);
            u[i] = ui;
            cost += gamma[i] * ui;
        }
        for (int r = 0; r < lp.p; ++r) {
            double sl = x[n + r], zs = z[n + r];
            active[lp.rowchk[r]] = !(sl > (o->tau_act > zs ? o->tau_act : zs));
        }
        if (trace_mask && k < trace_cap) {
            memcpy(trace_mask + (size_t)k * m, mask, sizeof(uint32_t) * m);
            double g = 0.0;
            for (int i = 0; i < n; ++i) g += gamma[i] * u[i];
            trace_obj[k] = g;
            trace_p[k] = lp.p;
            trace_ipm[k] = its;
        }
        lp_free(&lp);
        if (rc != 0) { s.status = rc; break; }
        /* Theorem 2b: the costs of successive LP solutions increase strictly. A decrease
           beyond the IPM's accuracy (relative to 1 + c^T x, the scale of its gap test; c^T x
           = gamma^T u - gneg) means a cut was replaced or dropped while it still bound the
           optimum: the decode stops with a failure flag instead of cycling. */
        if (last) break;
        if (cost < cost_prev - o->tau_cost * (1.0 + fabs(cost_prev - gneg))) { s.status = -5; break; }
        cost_prev2 = cost_prev;
        cost_prev = cost;
    }
    if (k == o->malp_max && s.status == 0) s.status = -3;
    /* output: integrality, hard decision of the LP solution, syndrome, objective */
    double fr = 0.0, g = 0.0;
    for (int i = 0; i < n; ++i) {
        double a = u[i] < 1.0 - u[i] ? u[i] : 1.0 - u[i];
        if (a > fr) fr = a;
        g += gamma[i] * u[i];
        if (fabs(u[i] - 0.5) <= o->tau_int) xhat[i] = gamma[i] >= 0.0 ? 0 : 1;
        else xhat[i] = u[i] > 0.5;
    }
    int syn = 0;
    for (int j = 0; j < m; ++j) {
        int par = 0;
        for (int t = rowptr[j]; t < rowptr[j + 1]; ++t) par ^= xhat[col[t]];
        syn |= par;
    }
    int integral = fr <= o->tau_int;
    if (s.status < 0) *flag = s.status;
    else if (integral && !syn) *flag = 1;
    else if (integral) *flag = -4;
    else *flag = 0;
    if (obj) *obj = g;
    if (u_out) memcpy(u_out, u, sizeof(double) * n);
    if (st) *st = s;
    free(mask); free(mask1); free(mask2); free(active); free(u); free(nb); free(x); free(z); free(y);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* ALP decoding (Algorithm 1): every LP keeps all cuts added so far; each iteration adds the  */
/* (at most one per check, Theorem 1) violated parity inequality of every check at the last  */
/* solution, found by Algorithm 2; box constraints are not searched (Theorem 2a). New cuts of */
/* an iteration follow the existing ones, in ascending check order. Same output, flags and   */
/* readings (box clamp, cost check) as orc_decode. trace_p[k] / trace_obj[k] / trace_ipm[k]: */
/* cuts, cost and IPM iterations of the k-th LP. cuts_out (optional, cap entries of          */
/* (check, V) pairs, 2 ints each) receives the final cut list; returns the number of cuts.    */
int orc_alp_decode(int m, int n, const int *rowptr, const int *col, const double *gamma,
                   const orc_opts *o, double *u_out, uint8_t *xhat, int *flag, double *obj,
                   orc_stats *st, double *trace_obj, int *trace_p, int *trace_ipm, int trace_cap,
                   int *cuts_out, int cuts_cap)
{
    int cap = 16 * m + 16, p = 0;
    int *chk = malloc(sizeof(int) * cap);
    uint32_t *Vs = malloc(sizeof(uint32_t) * cap);
    double *u = malloc(sizeof(double) * n);
    double *nb = malloc(sizeof(double) * 64);
    double *x = NULL, *z = NULL, *y = NULL;
    orc_stats s = {0, 0, 0, 0, 0};
    double gneg = 0.0;
    for (int i = 0; i < n; ++i) {
        u[i] = gamma[i] >= 0.0 ? 0.0 : 1.0;
        if (gamma[i] < 0.0) gneg += gamma[i];
    }
    double cost_prev = gneg;
    int k;
    for (k = 0; k < o->malp_max; ++k) {
        int added = 0;
        for (int j = 0; j < m; ++j) {
            int d = rowptr[j + 1] - rowptr[j];
            for (int t = 0; t < d; ++t) nb[t] = u[col[rowptr[j] + t]];
            uint32_t V;
            double lhs;
            if (orc_find_cut(d, nb, o->tau_viol, &V, &lhs)) {
                if (p == cap) {
                    cap *= 2;
                    chk = realloc(chk, sizeof(int) * cap);
                    Vs = realloc(Vs, sizeof(uint32_t) * cap);
                }
                chk[p] = j;
                Vs[p] = V;
                ++p;
                added = 1;
            }
        }
        if (!added) break;
        lp_t lp;
        lp_build_cuts(&lp, n, rowptr, col, gamma, p, chk, Vs);
        free(x); free(z); free(y);
        x = malloc(sizeof(double) * (n + p));
        z = malloc(sizeof(double) * (n + p));
        y = malloc(sizeof(double) * (p + 1));
        int its = 0;
        int rc = ipm_solve(&lp, o, x, y, z, &its);
        s.malp_iters++;
        s.ipm_iters += its;
        if (p > s.p_max) s.p_max = p;
        s.p_final = p;
        double cost = 0.0;
        for (int i = 0; i < n; ++i) {
            double ui = gamma[i] >= 0.0 ? x[i] : 1.0 - x[i];
            if (o->box_clamp) ui = ui < 0.0 ? 0.0 : (ui > 1.0 ? 1.0 : ui);
            u[i] = ui;
            cost += gamma[i] * ui;
        }
        if (trace_obj && k < trace_cap) {
            trace_obj[k] = cost;
            trace_p[k] = p;
            trace_ipm[k] = its;
        }
        lp_free(&lp);
        if (rc != 0) { s.status = rc; break; }
        if (cost < cost_prev - o->tau_cost * (1.0 + fabs(cost_prev - gneg))) { s.status = -5; break; }
        cost_prev = cost;
    }
    if (k == o->malp_max && s.status == 0) s.status = -3;
    double fr = 0.0, g = 0.0;
    for (int i = 0; i < n; ++i) {
        double a = u[i] < 1.0 - u[i] ? u[i] : 1.0 - u[i];
        if (a > fr) fr = a;
        g += gamma[i] * u[i];
        if (fabs(u[i] - 0.5) <= o->tau_int) xhat[i] = gamma[i] >= 0.0 ? 0 : 1;
        else xhat[i] = u[i] > 0.5;
    }
    int syn = 0;
    for (int j = 0; j < m; ++j) {
        int par = 0;
        for (int t = rowptr[j]; t < rowptr[j + 1]; ++t) par ^= xhat[col[t]];
        syn |= par;
    }
    int integral = fr <= o->tau_int;
    if (s.status < 0) *flag = s.status;
    else if (integral && !syn) *flag = 1;
    else if (integral) *flag = -4;
    else *flag = 0;
    if (obj) *obj = g;
    if (u_out) memcpy(u_out, u, sizeof(double) * n);
    if (st) *st = s;
    if (cuts_out)
        for (int r = 0; r < p && r < cuts_cap; ++r) { cuts_out[2 * r] = chk[r]; cuts_out[2 * r + 1] = (int)Vs[r]; }
    free(chk); free(Vs); free(u); free(nb); free(x); free(z); free(y);
    return p;
}

/* ------------------------------------------------------------------------------------ */
/* Test hooks: the LP of a cut set, one IPM solve, one Newton direction.                  */

/* Dense A [p*q], b [p], c [q] of the augmented LP of a cut set; returns p. */
int orc_lp_dense(int m, int n, const int *rowptr, const int *col, const double *gamma,
                 const uint32_t *mask, double *A, double *b, double *c)
{
    lp_t lp;
    lp_build(&lp, m, n, rowptr, col, gamma, mask);
    int p = lp.p, q = lp.q;
    if (A) {
        memset(A, 0, sizeof(double) * (size_t)p * q);
        for (int r = 0; r < p; ++r) {
            for (int t = lp.rptr[r]; t < lp.rptr[r + 1]; ++t) A[(size_t)r * q + lp.ridx[t]] = lp.rval[t];
            A[(size_t)r * q + n + r] = 1.0;
        }
    }
    if (b) memcpy(b, lp.b, sizeof(double) * p);
    if (c) memcpy(c, lp.c, sizeof(double) * q);
    lp_free(&lp);
    return p;
}

/* Solve the LP of a cut set by the IPM; x, z have q = n+p entries, y has p. */
int orc_ipm(int m, int n, const int *rowptr, const int *col, const double *gamma,
            const uint32_t *mask, const orc_opts *o, double *x, double *y, double *z, int *iters)
{
    lp_t lp;
    lp_build(&lp, m, n, rowptr, col, gamma, mask);
    int rc = ipm_solve(&lp, o, x, y, z, iters);
    lp_free(&lp);
    return rc;
}

/* One Newton direction at a given iterate (x, y, z) with a given mu. */
int orc_newton(int m, int n, const int *rowptr, const int *col, const double *gamma,
               const uint32_t *mask, const double *x, const double *y, const double *z, double mu,
               double *dx, double *dy, double *dz)
{
    lp_t lp;
    lp_build(&lp, m, n, rowptr, col, gamma, mask);
    int p = lp.p, q = lp.q;
    double *rb = malloc(sizeof(double) * (p + 1)), *rc = malloc(sizeof(double) * q);
    double *t1 = malloc(sizeof(double) * q), *t2 = malloc(sizeof(double) * q);
    double *Q = malloc(sizeof(double) * ((size_t)p * p + 1));
    double *dzq = malloc(sizeof(double) * q);
    newton(&lp, x, y, z, mu, dx, dy, dzq, rb, rc, Q, t1, t2);
    memcpy(dz, dzq, sizeof(double) * q);
    free(rb); free(rc); free(t1); free(t2); free(Q); free(dzq);
    lp_free(&lp);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Algorithm 7: column-wise greedy search for the maximum-weight triangular set.           */
/* Columns are numbered 0..n-1 (standard) and n+j (slack of check j); the weights w[]      */
/* have n+m entries and only columns of the LP (standard, or slack of a check with a cut)  */
/* are used. Key order: w descending, then column index ascending. A binary heap holds    */
/* the degree-1 columns (Sec. V-B); a column that lost its last row while waiting in the  */
/* heap is discarded when it surfaces.                                                     */
/* Outputs: pair[j] = column matched to row (check) j, -1 for checks without a cut;       */
/* order[k] = check eliminated at step k (k < p). Returns p.                               */
typedef struct { float w; int idx; } hkey;

static int key_gt(hkey a, hkey b) { return a.w > b.w || (a.w == b.w && a.idx < b.idx); }

static void heap_push(hkey *h, int *sz, hkey v)
{
    int i = (*sz)++;
    h[i] = v;
    while (i > 0) {
        int par = (i - 1) / 2;
        if (!key_gt(h[i], h[par])) break;
        hkey t = h[i]; h[i] = h[par]; h[par] = t;
        i = par;
    }
}

static hkey heap_pop(hkey *h, int *sz)
{
    hkey top = h[0];
    h[0] = h[--(*sz)];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, b = i;
        if (l < *sz && key_gt(h[l], h[b])) b = l;
        if (r < *sz && key_gt(h[r], h[b])) b = r;
        if (b == i) break;
        hkey t = h[i]; h[i] = h[b]; h[b] = t;
        i = b;
    }
    return top;
}

int orc_mts(int m, int n, const int *rowptr, const int *col, const uint8_t *hascut,
            const float *w, int *pair, int *order)
{
    int E = rowptr[m];
    /* column view of H restricted to rows with a cut */
    int *cptr = calloc(n + 1, sizeof(int));
    int *crow = malloc(sizeof(int) * (E + 1));
    for (int j = 0; j < m; ++j)
        if (hascut[j])
            for (int t = rowptr[j]; t < rowptr[j + 1]; ++t) cptr[col[t] + 1]++;
    for (int i = 0; i < n; ++i) cptr[i + 1] += cptr[i];
    int *fill = malloc(sizeof(int) * (n + 1));
    memcpy(fill, cptr, sizeof(int) * n);
    for (int j = 0; j < m; ++j)
        if (hascut[j])
            for (int t = rowptr[j]; t < rowptr[j + 1]; ++t) crow[fill[col[t]]++] = j;
    free(fill);
    int *deg = malloc(sizeof(int) * (n + m));      /* residual degree of each column */
    uint8_t *alive = malloc(m);                     /* row not yet eliminated */
    hkey *heap = malloc(sizeof(hkey) * (n + m + 1));
    int hs = 0, p = 0;
    for (int j = 0; j < m; ++j) { alive[j] = hascut[j]; pair[j] = -1; if (hascut[j]) ++p; }
    for (int i = 0; i < n; ++i) {
        deg[i] = cptr[i + 1] - cptr[i];
        if (deg[i] == 1) { hkey v = {w[i], i}; heap_push(heap, &hs, v); }
    }
    for (int j = 0; j < m; ++j) {
        deg[n + j] = hascut[j] ? 1 : 0;
        if (hascut[j]) { hkey v = {w[n + j], n + j}; heap_push(heap, &hs, v); }
    }
    int k = 0;
    while (k < p && hs > 0) {
        hkey top = heap_pop(heap, &hs);
        int c = top.idx;
        if (deg[c] != 1) continue;                 /* lost its last row while queued */
        /* the only remaining row of column c */
        int row = -1;
        if (c >= n) row = c - n;
        else
            for (int t = cptr[c]; t < cptr[c + 1]; ++t) if (alive[crow[t]]) { row = crow[t]; break; }
        pair[row] = c;
        order[k++] = row;
        /* eliminate the row: every column in it loses one degree */
        alive[row] = 0;
        deg[c] = 0;
        if (deg[n + row] > 0 && n + row != c) deg[n + row] = 0;   /* slack of the row dies */
        for (int t = rowptr[row]; t < rowptr[row + 1]; ++t) {
            int i = col[t];
            if (i == c || deg[i] <= 0) continue;
            deg[i]--;
            if (deg[i] == 1) { hkey v = {w[i], i}; heap_push(heap, &hs, v); }
        }
    }
    free(cptr); free(crow); free(deg); free(alive); free(heap);
    return k;
}

/* Column view (CSC) of H restricted to the checks that carry a cut, with the edge id of
   every entry so that coefficients stored per edge can be looked up from a column. */
typedef struct { int *cptr, *crow, *cedge; } colview;

static void colview_build(colview *cv, int m, int n, const int *rowptr, const int *col,
                          const uint8_t *hascut)
{
    int E = rowptr[m];
    cv->cptr = calloc(n + 1, sizeof(int));
    cv->crow = malloc(sizeof(int) * (E + 1));
    cv->cedge = malloc(sizeof(int) * (E + 1));
    for (int j = 0; j < m; ++j)
        if (hascut[j])
            for (int t = rowptr[j]; t < rowptr[j + 1]; ++t) cv->cptr[col[t] + 1]++;
    for (int i = 0; i < n; ++i) cv->cptr[i + 1] += cv->cptr[i];
    int *fill = malloc(sizeof(int) * (n + 1));
    memcpy(fill, cv->cptr, sizeof(int) * n);
    for (int j = 0; j < m; ++j)
        if (hascut[j])
            for (int t = rowptr[j]; t < rowptr[j + 1]; ++t) {
                int s = fill[col[t]]++;
                cv->crow[s] = j;
                cv->cedge[s] = t;
            }
    free(fill);
}

static void colview_free(colview *cv) { free(cv->cptr); free(cv->crow); free(cv->cedge); }

/* Dependency levels of the two triangular solves of M z = r (Sec. V):
   back-substitution A_M f1 = r solves row j for the column paired with it once every other
   preconditioner column in row j is known; forward substitution A_M^T z = f2 solves the
   column paired with row j once every other row of that column is known.
   lev_b[j] / lev_f[j] = length of the longest dependency chain below row j (0 = none);
   -1 for checks without a cut. Uses the elimination order of orc_mts. */
int orc_mts_levels(int m, int n, const int *rowptr, const int *col, const uint8_t *hascut,
                   const int *pair, const int *order, int p, int *lev_b, int *lev_f)
{
    colview cv;
    colview_build(&cv, m, n, rowptr, col, hascut);
    int *pairrow = malloc(sizeof(int) * (n + 1));  /* row paired with standard column i */
    for (int i = 0; i < n; ++i) pairrow[i] = -1;
    for (int j = 0; j < m; ++j) {
        lev_b[j] = -1; lev_f[j] = -1;
        if (hascut[j] && pair[j] >= 0 && pair[j] < n) pairrow[pair[j]] = j;
    }
    /* forward: the other rows of column pair[j] were eliminated earlier */
    for (int k = 0; k < p; ++k) {
        int j = order[k], c = pair[j], L = 0;
        if (c < n)
            for (int s = cv.cptr[c]; s < cv.cptr[c + 1]; ++s) {
                int jj = cv.crow[s];
                if (jj != j && lev_f[jj] + 1 > L) L = lev_f[jj] + 1;
            }
        lev_f[j] = L;
    }
    /* backward: the other preconditioner columns of row j are eliminated later */
    for (int k = p - 1; k >= 0; --k) {
        int j = order[k], L = 0;
        for (int t = rowptr[j]; t < rowptr[j + 1]; ++t) {
            int i = col[t];
            if (i == pair[j] || pairrow[i] < 0) continue;
            if (lev_b[pairrow[i]] + 1 > L) L = lev_b[pairrow[i]] + 1;
        }
        lev_b[j] = L;
    }
    free(pairrow);
    colview_free(&cv);
    return 0;
}

/* Algorithm 8: row-wise greedy search for the triangular set, with diagonal expansion.    */
/* Works on the residual matrix of the LP (rows = checks with a cut, columns = standard    */
/* columns with at least one such row and the slack of every such row). While a row of     */
/* residual degree 1 exists, the lowest-indexed one is matched with its only remaining     */
/* column, which is then removed; otherwise the remaining column of smallest key (w        */
/* ascending, then column index ascending) is removed unmatched. Rows left unmatched are   */
/* matched with their own slack column, in ascending order (diagonal expansion).           */
/* A_M is lower triangular in the returned order: the other matched columns of a row      */
/* belong to rows matched before it. Same outputs as orc_mts.                              */
int orc_mts_row2(int m, int n, const int *rowptr, const int *col, const uint8_t *hascut,
                 const float *w, int expand, int *pair, int *order);

int orc_mts_row(int m, int n, const int *rowptr, const int *col, const uint8_t *hascut,
                const float *w, int *pair, int *order)
{
    return orc_mts_row2(m, n, rowptr, col, hascut, w, 0, pair, order);
}

/* expand = 0: diagonal expansion; 1: triangular expansion -- the rows left unmatched are
   matched by the column-wise greedy search (Algorithm 7's rule: the degree-1 column of
   largest key, w descending then index ascending) on the columns whose rows are all
   unmatched (the matrix A-bar of Sec. V-B), after the rows of the row-wise phase. */
int orc_mts_row2(int m, int n, const int *rowptr, const int *col, const uint8_t *hascut,
                 const float *w, int expand, int *pair, int *order)
{
    colview cv;
    colview_build(&cv, m, n, rowptr, col, hascut);
    uint8_t *alive = calloc(n + m, 1);     /* column still in the residual matrix */
    int *rdeg = calloc(m, sizeof(int));    /* remaining columns of each row */
    int k = 0, live = 0;
    for (int i = 0; i < n; ++i) alive[i] = cv.cptr[i + 1] > cv.cptr[i];
    for (int j = 0; j < m; ++j) {
        pair[j] = -1;
        if (!hascut[j]) continue;
        alive[n + j] = 1;
        rdeg[j] = rowptr[j + 1] - rowptr[j] + 1;
        ++live;
    }
    while (live > 0) {
        int jr = -1;
        for (int j = 0; j < m; ++j)
            if (hascut[j] && pair[j] < 0 && rdeg[j] == 1) { jr = j; break; }
        int c = -1;
        if (jr >= 0) {
            /* the only remaining column of row jr */
            if (alive[n + jr]) c = n + jr;
            for (int t = rowptr[jr]; t < rowptr[jr + 1]; ++t) if (alive[col[t]]) c = col[t];
            pair[jr] = c;
            order[k++] = jr;
        } else {
            for (int i = 0; i < n + m; ++i) {
                if (!alive[i]) continue;
                if (c < 0 || w[i] < w[c]) c = i;     /* ascending index breaks ties */
            }
            if (c < 0) break;
        }
        /* remove column c: each of its rows loses one degree */
        alive[c] = 0;
        if (c >= n) {
            if (--rdeg[c - n] == 0) --live;
        } else {
            for (int s2 = cv.cptr[c]; s2 < cv.cptr[c + 1]; ++s2)
                if (--rdeg[cv.crow[s2]] == 0) --live;
        }
    }
    if (expand == 1) {
        /* A-bar: columns all of whose LP rows are unmatched; greedy by columns over it */
        int *deg = calloc(n + m, sizeof(int));      /* live rows of each A-bar column, -1 outside */
        uint8_t *live = calloc(m, 1);
        int left = 0;
        for (int j = 0; j < m; ++j) if (hascut[j] && pair[j] < 0) { live[j] = 1; ++left; }
        for (int i = 0; i < n; ++i) {
            int d = cv.cptr[i + 1] - cv.cptr[i];
            for (int s2 = cv.cptr[i]; s2 < cv.cptr[i + 1]; ++s2) if (!live[cv.crow[s2]]) d = -1;
            deg[i] = d > 0 ? d : -1;
        }
        for (int j = 0; j < m; ++j) deg[n + j] = live[j] ? 1 : -1;
        while (left > 0) {
            int c = -1;
            for (int i = 0; i < n + m; ++i)
                if (deg[i] == 1 && (c < 0 || w[i] > w[c])) c = i;   /* ascending index breaks ties */
            if (c < 0) break;
            int row = -1;
            if (c >= n) row = c - n;
            else
                for (int s2 = cv.cptr[c]; s2 < cv.cptr[c + 1]; ++s2) if (live[cv.crow[s2]]) row = cv.crow[s2];
            pair[row] = c;
            order[k++] = row;
            live[row] = 0;
            --left;
            deg[c] = -1;
            if (c != n + row) deg[n + row] = -1;
            for (int t = rowptr[row]; t < rowptr[row + 1]; ++t)
                if (col[t] != c && deg[col[t]] > 0) deg[col[t]]--;
        }
        free(deg); free(live);
    }
    for (int j = 0; j < m; ++j)
        if (hascut[j] && pair[j] < 0) { pair[j] = n + j; order[k++] = j; }
    free(alive); free(rdeg);
    colview_free(&cv);
    return k;
}

/* Algorithm 5 (Triangulation Step) on a column set S of the LP's A (inS[c] != 0; c < n a    */
/* standard column, c = n + j the slack of check j, which must carry a cut). Peeling: a row    */
/* with exactly one remaining column of S is matched with it, and that column leaves; A_S     */
/* is lower triangular in matching order. The paper lets any degree-1 row go next; here the   */
/* peeling runs in rounds: the rows of degree 1 at the start of a round, in ascending order,  */
/* each take their column unless an earlier row of the round has taken it. Rows that reach    */
/* degree 1 during a round wait for the next one. Success iff every column of S is matched:  */
/* returns the number matched; pair[j] = column of row j (-1 unmatched), order[k] = row      */
/* matched k-th.                                                                             */
int orc_triangulate(int m, int n, const int *rowptr, const int *col, const uint8_t *hascut,
                    const uint8_t *inS, int *pair, int *order)
{
    colview cv;
    colview_build(&cv, m, n, rowptr, col, hascut);
    int *rdeg = calloc(m, sizeof(int));
    uint8_t *gone = calloc(n + m, 1);          /* column of S already matched */
    int *round_rows = malloc(sizeof(int) * (m + 1));
    int s = 0, k = 0;
    for (int c = 0; c < n + m; ++c) s += inS[c] != 0;
    for (int j = 0; j < m; ++j) {
        pair[j] = -1;
        if (!hascut[j]) continue;
        int d = inS[n + j] ? 1 : 0;
        for (int t = rowptr[j]; t < rowptr[j + 1]; ++t) d += inS[col[t]] != 0;
        rdeg[j] = d;
    }
    for (;;) {
        int nr = 0;
        for (int j = 0; j < m; ++j)
            if (hascut[j] && pair[j] < 0 && rdeg[j] == 1) round_rows[nr++] = j;
        if (nr == 0) break;
        for (int a = 0; a < nr; ++a) {
            int j = round_rows[a], c = -1;
            if (inS[n + j] && !gone[n + j]) c = n + j;
            for (int t = rowptr[j]; t < rowptr[j + 1]; ++t)
                if (inS[col[t]] && !gone[col[t]]) c = col[t];
            if (c < 0) continue;                  /* its column went to an earlier row */
            pair[j] = c;
            order[k++] = j;
            gone[c] = 1;
            if (c >= n) rdeg[c - n]--;
            else
                for (int t = cv.cptr[c]; t < cv.cptr[c + 1]; ++t) rdeg[cv.crow[t]]--;
        }
    }
    free(rdeg); free(gone); free(round_rows);
    colview_free(&cv);
    (void)s;
    return k;
}

/* Algorithm 6: incremental greedy search for the triangular set. The LP's columns (all n    */
/* standard columns and the slack of every check with a cut) in the order of the key (w      */
/* descending, then column index ascending); each is added to M when M with it still passes  */
/* the Triangulation Step, until M has p columns. The pairing and order are those of the     */
/* Triangulation Step on the final M (A_M lower triangular in that order). Returns p.        */
typedef struct { float w; int idx; } ckey;

static int ckey_cmp(const void *a, const void *b)
{
    const ckey *x = a, *y = b;
    if (x->w != y->w) return x->w > y->w ? -1 : 1;
    return x->idx - y->idx;
}

int orc_mts_inc(int m, int n, const int *rowptr, const int *col, const uint8_t *hascut,
                const float *w, int *pair, int *order, int *calls)
{
    int p = 0, q = 0;
    for (int j = 0; j < m; ++j) p += hascut[j] != 0;
    ckey *keys = malloc(sizeof(ckey) * (n + m + 1));
    for (int c = 0; c < n + m; ++c)
        if (c < n || hascut[c - n]) { keys[q].w = w[c]; keys[q].idx = c; ++q; }
    qsort(keys, q, sizeof(ckey), ckey_cmp);
    uint8_t *inS = calloc(n + m, 1);
    int msz = 0, nc = 0;
    for (int t = 0; t < q && msz < p; ++t) {
        inS[keys[t].idx] = 1;
        ++nc;
        if (orc_triangulate(m, n, rowptr, col, hascut, inS, pair, order) == msz + 1) ++msz;
        else inS[keys[t].idx] = 0;
    }
    int k = orc_triangulate(m, n, rowptr, col, hascut, inS, pair, order);
    if (calls) *calls = nc + 1;
    free(keys); free(inS);
    return k;
}

/* Dependency levels of the two triangular solves for any triangular set (Sec. V): lev_b[j]
   = 1 + the largest lev_b over the rows matched with the other preconditioner columns of
   row j (0 without such rows); lev_f[j] = 1 + the largest lev_f over the other rows of the
   column matched with row j. Longest chains by memoised depth-first search, without
   assuming which way the dependencies point. -1 for checks without a cut. */
static int lvl_b(int j, int n, const int *rowptr, const int *col, const int *pair, const int *pairrow, int *lev)
{
    if (lev[j] >= 0) return lev[j];
    int L = 0;
    for (int t = rowptr[j]; t < rowptr[j + 1]; ++t) {
        int i = col[t];
        if (i == pair[j] || pairrow[i] < 0) continue;
        int v = lvl_b(pairrow[i], n, rowptr, col, pair, pairrow, lev) + 1;
        if (v > L) L = v;
    }
    return lev[j] = L;
}

static int lvl_f(int j, int n, const colview *cv, const int *pair, int *lev)
{
    if (lev[j] >= 0) return lev[j];
    int L = 0, c = pair[j];
    if (c < n)
        for (int s = cv->cptr[c]; s < cv->cptr[c + 1]; ++s) {
            int jj = cv->crow[s];
            if (jj == j) continue;
            int v = lvl_f(jj, n, cv, pair, lev) + 1;
            if (v > L) L = v;
        }
    return lev[j] = L;
}

int orc_mts_levels_any(int m, int n, const int *rowptr, const int *col, const uint8_t *hascut,
                       const int *pair, int *lev_b, int *lev_f)
{
    colview cv;
    colview_build(&cv, m, n, rowptr, col, hascut);
    int *pairrow = malloc(sizeof(int) * (n + 1));
    for (int i = 0; i < n; ++i) pairrow[i] = -1;
    for (int j = 0; j < m; ++j) {
        lev_b[j] = -1; lev_f[j] = -1;
        if (hascut[j] && pair[j] >= 0 && pair[j] < n) pairrow[pair[j]] = j;
    }
    for (int j = 0; j < m; ++j)
        if (hascut[j]) { lvl_b(j, n, rowptr, col, pair, pairrow, lev_b); lvl_f(j, n, &cv, pair, lev_f); }
    free(pairrow);
    colview_free(&cv);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Algorithm 4 (PCG) in FP64 on (A D^2 A^T) y = w with the triangular preconditioner of    */
/* Sec. V built by Algorithm 7 from the weights wkey (float d^2). Vectors live in check    */
/* space (length m; entries of checks without a cut are ignored and returned as 0).        */
/* d2 has n+m entries (standard, then slack of check j at n+j). The preconditioner solve   */
/* is A_M f1 = r, f2 = D_M^-2 f1, A_M^T z = f2, in elimination order. Stops when          */
/* ||r|| <= tol ||w||, at maxit, or when h^T l <= 0. Returns the iteration count;          */
/* resid[i] (optional, maxit+1 entries) receives ||r^i|| / ||w||.                          */
typedef struct {
    int m, n, p;
    const int *rowptr, *col;
    const uint8_t *hascut;
    const double *sg;         /* A entry per edge of H (0 off the LP) */
    const double *d2;
    colview cv;
    int *pair, *order, *pairrow;
    double *F;                /* f1, stored at the row paired with each column */
} pcg_ctx;

/* l = (A D^2 A^T) h, via t = D^2 A^T h over standard columns */
static void pcg_Q(const pcg_ctx *P, const double *h, double *t, double *l)
{
    for (int i = 0; i < P->n; ++i) {
        double s = 0.0;
        for (int k = P->cv.cptr[i]; k < P->cv.cptr[i + 1]; ++k) s += P->sg[P->cv.cedge[k]] * h[P->cv.crow[k]];
        t[i] = P->d2[i] * s;
    }
    for (int j = 0; j < P->m; ++j) {
        if (!P->hascut[j]) { l[j] = 0.0; continue; }
        double s = P->d2[P->n + j] * h[j];
        for (int e = P->rowptr[j]; e < P->rowptr[j + 1]; ++e) s += P->sg[e] * t[P->col[e]];
        l[j] = s;
    }
}

/* A entry of (row j, standard column c) */
static double pcg_aent(const pcg_ctx *P, int j, int c)
{
    for (int e = P->rowptr[j]; e < P->rowptr[j + 1]; ++e) if (P->col[e] == c) return P->sg[e];
    return 0.0;
}

/* zz = M^-1 r with M = A_M D_M^2 A_M^T */
static void pcg_psolve(const pcg_ctx *P, const double *r, double *zz)
{
    int n = P->n;
    for (int j = 0; j < P->m; ++j) zz[j] = 0.0;
    /* A_M f1 = r: rows in reverse elimination order */
    for (int k = P->p - 1; k >= 0; --k) {
        int j = P->order[k], c = P->pair[j];
        double s = r[j];
        for (int e = P->rowptr[j]; e < P->rowptr[j + 1]; ++e) {
            int i = P->col[e];
            if (i != c && P->pairrow[i] >= 0) s -= P->sg[e] * P->F[P->pairrow[i]];
        }
        P->F[j] = s / (c >= n ? 1.0 : pcg_aent(P, j, c));
    }
    /* f2 = D_M^-2 f1, then A_M^T z = f2: rows in elimination order */
    for (int k = 0; k < P->p; ++k) {
        int j = P->order[k], c = P->pair[j];
        double s = P->F[j] / P->d2[c];
        if (c < n) {
            for (int t = P->cv.cptr[c]; t < P->cv.cptr[c + 1]; ++t) {
                int jj = P->cv.crow[t];
                if (jj != j) s -= P->sg[P->cv.cedge[t]] * zz[jj];
            }
            s /= pcg_aent(P, j, c);
        }
        zz[j] = s;
    }
}

int orc_pcg(int m, int n, const int *rowptr, const int *col, const double *gamma,
            const uint32_t *mask, const double *d2, const float *wkey, const double *w,
            double tol, int maxit, int use_precond, double *y, double *resid)
{
    int E = rowptr[m];
    uint8_t *hascut = malloc(m);
    double *sg = malloc(sizeof(double) * (E + 1));
    for (int j = 0; j < m; ++j) {
        hascut[j] = mask[j] != 0;
        for (int e = rowptr[j]; e < rowptr[j + 1]; ++e) {
            int k = e - rowptr[j], i = col[e];
            int s = ((mask[j] >> k) & 1u) ? 1 : -1;
            sg[e] = hascut[j] ? (double)((gamma[i] >= 0.0 ? 1 : -1) * s) : 0.0;
        }
    }
    pcg_ctx P;
    P.m = m; P.n = n; P.rowptr = rowptr; P.col = col; P.hascut = hascut; P.sg = sg; P.d2 = d2;
    colview_build(&P.cv, m, n, rowptr, col, hascut);
    P.pair = malloc(sizeof(int) * m);
    P.order = malloc(sizeof(int) * (m + 1));
    P.pairrow = malloc(sizeof(int) * (n + 1));
    P.F = calloc(m, sizeof(double));
    P.p = orc_mts(m, n, rowptr, col, hascut, wkey, P.pair, P.order);
    for (int i = 0; i < n; ++i) P.pairrow[i] = -1;
    for (int j = 0; j < m; ++j) if (P.pair[j] >= 0 && P.pair[j] < n) P.pairrow[P.pair[j]] = j;
    double *r = calloc(m, sizeof(double)), *zz = calloc(m, sizeof(double));
    double *h = calloc(m, sizeof(double)), *l = calloc(m, sizeof(double));
    double *t = calloc(n + 1, sizeof(double));
    /* Algorithm 4 with initial guess 0, so r^0 = w */
    double nw = 0.0;
    for (int j = 0; j < m; ++j) { y[j] = 0.0; r[j] = hascut[j] ? w[j] : 0.0; nw += r[j] * r[j]; }
    nw = sqrt(nw);
    if (resid) resid[0] = 1.0;
    int it = 0;
    if (nw > 0.0) {
        if (use_precond) pcg_psolve(&P, r, zz);
        else for (int j = 0; j < m; ++j) zz[j] = r[j];
        for (int j = 0; j < m; ++j) h[j] = zz[j];
        double rz = dot(r, zz, m);
        while (it < maxit) {
            pcg_Q(&P, h, t, l);
            double hl = dot(h, l, m);
            if (!(hl > 0.0)) break;
            double alpha = rz / hl, nr = 0.0;
            for (int j = 0; j < m; ++j) { y[j] += alpha * h[j]; r[j] -= alpha * l[j]; nr += r[j] * r[j]; }
            ++it;
            nr = sqrt(nr);
            if (resid) resid[it] = nr / nw;
            if (nr <= tol * nw) break;
            if (use_precond) pcg_psolve(&P, r, zz);
            else for (int j = 0; j < m; ++j) zz[j] = r[j];
            double rz2 = dot(r, zz, m);
            double nu = rz2 / rz;
            rz = rz2;
            for (int j = 0; j < m; ++j) h[j] = zz[j] + nu * h[j];
        }
    }
    free(hascut); free(sg); colview_free(&P.cv); free(P.pair); free(P.order); free(P.pairrow);
    free(P.F); free(r); free(zz); free(h); free(l); free(t);
    return it;
}

/* Exact solve of the same system by Cholesky, for tests (check-space vectors). */
int orc_normal_solve(int m, int n, const int *rowptr, const int *col, const double *gamma,
                     const uint32_t *mask, const double *d2, const double *w, double *y)
{
    lp_t lp;
    lp_build(&lp, m, n, rowptr, col, gamma, mask);
    int p = lp.p;
    double *d2q = malloc(sizeof(double) * (lp.q + 1));
    for (int i = 0; i < n; ++i) d2q[i] = d2[i];
    for (int r = 0; r < p; ++r) d2q[n + r] = d2[n + lp.rowchk[r]];
    double *Q = malloc(sizeof(double) * ((size_t)p * p + 1));
    double *wr = malloc(sizeof(double) * (p + 1)), *yr = malloc(sizeof(double) * (p + 1));
    for (int r = 0; r < p; ++r) wr[r] = w[lp.rowchk[r]];
    normal_matrix(&lp, d2q, Q);
    cholesky(Q, p);
    chol_solve(Q, p, wr, yr);
    for (int j = 0; j < m; ++j) y[j] = 0.0;
    for (int r = 0; r < p; ++r) y[lp.rowchk[r]] = yr[r];
    free(d2q); free(Q); free(wr); free(yr);
    lp_free(&lp);
    return p;
}
