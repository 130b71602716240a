/*
 * dpf_oracle.c -- plain, slow FP64 CPU reference for Differentiable Power-Flow.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness oracle against which
 * the GPU library is checked; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may call it.  It shares no code, header, table
 * or constant with the GPU path.
 *
 * Everything follows the paper's statement of the method (arXiv 2603.28203):
 *   - power balance S_calc = V .* conj(Y_bus V)                 (Sec. 2.1, Eq. powerbalance)
 *   - bus-type specification PV / PQ / slack                    (Sec. 2.1, Eq. pf_equation_full)
 *   - least-squares form over |V|_pq and theta_{pv,pq}          (Sec. 2.1, Eq. pf_optimization_problem)
 *   - MSE loss over out = [P_calc[pv,pq], Q_calc[pq]]           (Algorithm 1, forward pass)
 *   - gradient = J^T F without storing J                        (Sec. 5.1-5.3)
 *   - the NR partial derivatives dS/d|V|, dS/dtheta             (Algorithm 2, partial derivatives)
 *   - Adam (Kingma & Ba, bias corrected) with per-case stop test (Algorithm 1, optimizer loop)
 *
 * Readings where the paper is silent (branch model, loss normalisation, stop
 * test, Adam constants, scheduler semantics) are listed in the design notes;
 * each function below states the one it uses.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fcx-limited-range -fopenmp -fPIC -shared
 * (-fcx-limited-range makes complex multiply the textbook (ac-bd)+(ad+bc)i
 * without the Inf/NaN recovery branch; -ffp-contract=off keeps every product
 * and sum separately rounded in the written order.)
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define BUS_PQ 0
#define BUS_PV 1
#define BUS_SLACK 2

/* ------------------------------------------------------------------ Y-bus */

typedef struct {
    int32_t row, col;
    int32_t order; /* position of the contribution, used to sum in a fixed order */
    double complex val;
} triplet_t;

static int cmp_triplet(const void *pa, const void *pb)
{
    const triplet_t *a = (const triplet_t *)pa, *b = (const triplet_t *)pb;
    if (a->row != b->row) return a->row < b->row ? -1 : 1;
    if (a->col != b->col) return a->col < b->col ? -1 : 1;
    return a->order < b->order ? -1 : (a->order > b->order);
}

/*
 * Bus admittance matrix from pi-model branches (Sec. 2.1; the paper defers the
 * branch model to the MATPOWER manual).  Reading used: series admittance
 * y = 1/(r + jx), total charging b split b/2 to each end, no taps, no phase
 * shifters, no bus shunts:
 *     Y_ff += y + j b/2,  Y_tt += y + j b/2,  Y_ft += -y,  Y_tf += -y.
 * Parallel branches are summed; every diagonal entry is stored, even if zero.
 * Branch `skip` (or -1 for none) is left out entirely -- the N-1 outage case.
 * Output: CSR with rows sorted by column; contributions to one entry are added
 * in branch order, starting from zero.
 * Returns nnz, -1 on invalid input, -2 if cap is too small.
 */
int orc_ybus(int32_t n_bus, int32_t n_branch, const int32_t *f, const int32_t *t,
             const double *r, const double *x, const double *b, int32_t skip,
             int32_t cap, int32_t *row_ptr, int32_t *col, double complex *val)
{
    if (n_bus <= 0 || n_branch < 0) return -1;
    int32_t ntrip = n_bus + 4 * n_branch;
    triplet_t *tr = (triplet_t *)malloc(sizeof(triplet_t) * (size_t)(ntrip > 0 ? ntrip : 1));
    if (!tr) return -1;
    int32_t k = 0;
    for (int32_t i = 0; i < n_bus; ++i) {
        tr[k].row = i; tr[k].col = i; tr[k].order = k; tr[k].val = 0.0; ++k;
    }
    for (int32_t e = 0; e < n_branch; ++e) {
        if (f[e] < 0 || f[e] >= n_bus || t[e] < 0 || t[e] >= n_bus || f[e] == t[e] ||
            (r[e] == 0.0 && x[e] == 0.0)) {
            free(tr);
            return -1;
        }
        if (e == skip) continue;
        double complex y = 1.0 / (r[e] + I * x[e]);
        double complex ysh = I * (b[e] / 2.0);
        tr[k].row = f[e]; tr[k].col = f[e]; tr[k].order = k; tr[k].val = y + ysh; ++k;
        tr[k].row = t[e]; tr[k].col = t[e]; tr[k].order = k; tr[k].val = y + ysh; ++k;
        tr[k].row = f[e]; tr[k].col = t[e]; tr[k].order = k; tr[k].val = -y; ++k;
        tr[k].row = t[e]; tr[k].col = f[e]; tr[k].order = k; tr[k].val = -y; ++k;
    }
    qsort(tr, (size_t)k, sizeof(triplet_t), cmp_triplet);
    int32_t nnz = 0;
    for (int32_t i = 0; i <= n_bus; ++i) row_ptr[i] = 0;
    for (int32_t q = 0; q < k; ++q) {
        if (q > 0 && tr[q].row == tr[q - 1].row && tr[q].col == tr[q - 1].col) {
            val[nnz - 1] += tr[q].val;
            continue;
        }
        if (nnz >= cap) { free(tr); return -2; }
        col[nnz] = tr[q].col;
        val[nnz] = tr[q].val;
        row_ptr[tr[q].row + 1] += 1;
        ++nnz;
    }
    for (int32_t i = 0; i < n_bus; ++i) row_ptr[i + 1] += row_ptr[i];
    free(tr);
    return nnz;
}

/* ------------------------------------------------------------ power balance */

/* Polar to rectangular: V_i = |V_i| e^{j theta_i} (Sec. 4, polar form). */
void orc_polar(int32_t n, const double *vm, const double *va, double complex *V)
{
    for (int32_t i = 0; i < n; ++i) V[i] = vm[i] * (cos(va[i]) + I * sin(va[i]));
}

/* Current injections I = Y V, each row summed in stored (column) order. */
void orc_current(int32_t n, const int32_t *rp, const int32_t *ci, const double complex *yv,
                 const double complex *V, double complex *Icur)
{
    for (int32_t i = 0; i < n; ++i) {
        double complex acc = 0.0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) acc += yv[q] * V[ci[q]];
        Icur[i] = acc;
    }
}

/* Complex power mismatch dS = V .* conj(Y V) - S_spec (Eq. powerbalance). */
void orc_mismatch(int32_t n, const int32_t *rp, const int32_t *ci, const double complex *yv,
                  const double *vm, const double *va, const double complex *s_spec,
                  double complex *dS)
{
    double complex *V = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *Ic = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    orc_polar(n, vm, va, V);
    orc_current(n, rp, ci, yv, V, Ic);
    for (int32_t i = 0; i < n; ++i) dS[i] = V[i] * conj(Ic[i]) - s_spec[i];
    free(V);
    free(Ic);
}

/* Number of residuals m = |pv| + 2|pq| (length of `out` in Algorithm 1). */
int32_t orc_residual_count(int32_t n, const int8_t *bus_type)
{
    int32_t m = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (bus_type[i] == BUS_PV) m += 1;
        else if (bus_type[i] == BUS_PQ) m += 2;
    }
    return m;
}

/*
 * Loss and convergence measure from a mismatch vector.
 * out - target = [dP[pv,pq], dQ[pq]] (Algorithm 1), so
 *   loss = MSE = (1/m) sum over those entries of the squared residual,
 *   mu   = largest absolute entry (the stop test's max|dS| in pu).
 * Returns loss; *mu receives mu.  NaN propagates into both.
 */
double orc_loss_from_mismatch(int32_t n, const int8_t *bus_type, const double complex *dS,
                              double *mu)
{
    int32_t m = orc_residual_count(n, bus_type);
    double sum = 0.0, mx = 0.0;
    int bad = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (bus_type[i] == BUS_SLACK) continue;
        double p = creal(dS[i]);
        sum += p * p;
        if (!(fabs(p) <= mx)) { if (isnan(p)) bad = 1; else mx = fabs(p); }
        if (bus_type[i] == BUS_PQ) {
            double q = cimag(dS[i]);
            sum += q * q;
            if (!(fabs(q) <= mx)) { if (isnan(q)) bad = 1; else mx = fabs(q); }
        }
    }
    *mu = bad ? NAN : mx;
    return m > 0 ? sum / (double)m : 0.0;
}

/*
 * NR partial derivatives of S_calc with respect to |V| and theta, stored in
 * the sparsity pattern of Y (Algorithm 2, "partial derivatives"):
 *   dS_i/d|V_j| = V_i conj(Y_ij) conj(V_j) / |V_j|                         (i != j)
 *   dS_i/d|V_i| = V_i/|V_i| conj(I_i) + V_i conj(Y_ii) conj(V_i) / |V_i|
 *   dS_i/dth_j  = -j V_i conj(Y_ij) conj(V_j)                              (i != j)
 *   dS_i/dth_i  =  j V_i conj(I_i) - j V_i conj(Y_ii) conj(V_i)
 * with I = Y V.  Entry q of each output belongs to (row i, column ci[q]).
 */
void orc_dS_dV(int32_t n, const int32_t *rp, const int32_t *ci, const double complex *yv,
               const double *vm, const double *va, double complex *dS_dvm,
               double complex *dS_dva)
{
    double complex *V = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *Ic = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    orc_polar(n, vm, va, V);
    orc_current(n, rp, ci, yv, V, Ic);
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            int32_t j = ci[q];
            double complex term = V[i] * conj(yv[q]) * conj(V[j]);
            if (j != i) {
                dS_dvm[q] = term / vm[j];
                dS_dva[q] = -I * term;
            } else {
                dS_dvm[q] = V[i] / vm[i] * conj(Ic[i]) + term / vm[i];
                dS_dva[q] = I * V[i] * conj(Ic[i]) - I * term;
            }
        }
    }
    free(V);
    free(Ic);
}

/*
 * Gradient of the MSE loss, dL/dx = (2/m) J_f^T f (Sec. 5.1: gradient descent
 * projects the mismatch back through J^T), where f = [dP[pv,pq], dQ[pq]] and
 * J_f holds the rows of the Algorithm 2 partial derivatives for those
 * residuals.  J_f is never stored: each row's entries are formed and applied
 * to f at once.  Only learnable coordinates get a gradient (|V| at PQ buses,
 * theta at PV and PQ buses); all others are set to 0.
 * Returns the loss; *mu receives the max-abs residual.
 */
double orc_loss_grad(int32_t n, const int32_t *rp, const int32_t *ci, const double complex *yv,
                     const int8_t *bus_type, const double *vm, const double *va,
                     const double complex *s_spec, double *g_vm, double *g_va, double *mu)
{
    int32_t nnz = rp[n];
    double complex *dvm = (double complex *)malloc(sizeof(double complex) * (size_t)(nnz > 0 ? nnz : 1));
    double complex *dva = (double complex *)malloc(sizeof(double complex) * (size_t)(nnz > 0 ? nnz : 1));
    double complex *dS = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    orc_dS_dV(n, rp, ci, yv, vm, va, dvm, dva);
    orc_mismatch(n, rp, ci, yv, vm, va, s_spec, dS);
    double loss = orc_loss_from_mismatch(n, bus_type, dS, mu);
    int32_t m = orc_residual_count(n, bus_type);
    double scale = m > 0 ? 2.0 / (double)m : 0.0;
    for (int32_t j = 0; j < n; ++j) { g_vm[j] = 0.0; g_va[j] = 0.0; }
    for (int32_t i = 0; i < n; ++i) {
        if (bus_type[i] == BUS_SLACK) continue;            /* no residual rows at the slack */
        double fP = creal(dS[i]);
        double fQ = bus_type[i] == BUS_PQ ? cimag(dS[i]) : 0.0; /* Q row only at PQ */
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            int32_t j = ci[q];
            g_va[j] += scale * (fP * creal(dva[q]) + fQ * cimag(dva[q]));
            g_vm[j] += scale * (fP * creal(dvm[q]) + fQ * cimag(dvm[q]));
        }
    }
    for (int32_t j = 0; j < n; ++j) {
        if (bus_type[j] != BUS_PQ) g_vm[j] = 0.0;      /* |V| learnable at PQ only */
        if (bus_type[j] == BUS_SLACK) g_va[j] = 0.0;   /* theta learnable at PV, PQ */
    }
    free(dvm);
    free(dva);
    free(dS);
    return loss;
}

/* ------------------------------------------------------- parameter gradient */

/*
 * Gradient of the loss with respect to the simulation parameters (Sec. 1 and
 * Sec. 2.3: gradients propagate from the power mismatch to the parameters of
 * the simulation, which can then be identified by gradient descent).
 * Parameters: each branch's r, x, b (pi model, Sec. 2.1 via Y) and the
 * specified injections S_spec.  Forward mode, one parameter at a time: a branch
 * parameter p changes only the four entries of Y that the branch stamps,
 *   dY_ff = dY_tt = dy + j db/2,  dY_ft = dY_tf = -dy,  y = 1/(r + jx),
 *   dy/dr = -y^2,  dy/dx = -j y^2,
 * so dI = dY V is nonzero at f and t only, dS_i = V_i conj(dI_i) there, and
 *   dL = (2/m) sum_{i in {f,t}} (r^P_i Re dS_i + r^Q_i Im dS_i).
 * For S_spec: d dS_i / d S_i = -1, so dL/dRe S_i = -(2/m) r^P_i and
 * dL/dIm S_i = -(2/m) r^Q_i (returned as one complex number per bus).
 * Branch `skip` (an N-1 outage, or -1) is absent from Y: its gradients are 0.
 * The residuals come from Y given in CSR (which must already exclude `skip`).
 */
void orc_param_grad(int32_t n, int32_t n_branch, const int32_t *from, const int32_t *to,
                    const double *r, const double *x, const double *b, int32_t skip,
                    const int32_t *rp, const int32_t *ci, const double complex *yv,
                    const int8_t *bus_type, const double *vm, const double *va,
                    const double complex *s_spec, double *g_r, double *g_x, double *g_b,
                    double complex *g_s)
{
    double complex *V = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    double complex *dS = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    orc_polar(n, vm, va, V);
    orc_mismatch(n, rp, ci, yv, vm, va, s_spec, dS);
    int32_t m = orc_residual_count(n, bus_type);
    double k = m > 0 ? 2.0 / (double)m : 0.0;
    /* masked residuals r^P, r^Q per bus */
    double *rP = (double *)calloc((size_t)n, sizeof(double));
    double *rQ = (double *)calloc((size_t)n, sizeof(double));
    for (int32_t i = 0; i < n; ++i) {
        if (bus_type[i] != BUS_SLACK) rP[i] = creal(dS[i]);
        if (bus_type[i] == BUS_PQ) rQ[i] = cimag(dS[i]);
        if (g_s) g_s[i] = -k * rP[i] - I * (k * rQ[i]);
    }
    for (int32_t e = 0; e < n_branch; ++e) {
        double gr = 0.0, gx = 0.0, gb = 0.0;
        if (e != skip && from[e] != to[e]) {
            int32_t f = from[e], t = to[e];
            double complex y = 1.0 / (r[e] + I * x[e]);
            /* dY stamps per unit change of r, x and b */
            double complex dy_dp[3] = {-y * y, -I * y * y, 0.0};
            double complex dsh_dp[3] = {0.0, 0.0, 0.5 * I};
            double out3[3];
            for (int p = 0; p < 3; ++p) {
                double complex dI_f = (dy_dp[p] + dsh_dp[p]) * V[f] - dy_dp[p] * V[t];
                double complex dI_t = (dy_dp[p] + dsh_dp[p]) * V[t] - dy_dp[p] * V[f];
                double complex dS_f = V[f] * conj(dI_f), dS_t = V[t] * conj(dI_t);
                out3[p] = k * (rP[f] * creal(dS_f) + rQ[f] * cimag(dS_f) +
                               rP[t] * creal(dS_t) + rQ[t] * cimag(dS_t));
            }
            gr = out3[0];
            gx = out3[1];
            gb = out3[2];
        }
        if (g_r) g_r[e] = gr;
        if (g_x) g_x[e] = gx;
        if (g_b) g_b[e] = gb;
    }
    free(V);
    free(dS);
    free(rP);
    free(rQ);
}

/* ------------------------------------------------------------- Adam solve */

typedef struct {
    double lr, beta1, beta2, eps, tol;
    int32_t max_iter;
    /* learning-rate schedule: 0 constant, 1 reduce-on-plateau, 2 step */
    int32_t sched;
    double factor;      /* plateau: multiply lr by this on a plateau; step: gamma */
    int32_t patience;   /* plateau: bad iterations tolerated; step: step size    */
    double threshold;   /* plateau: relative improvement needed                  */
    int32_t cooldown;   /* plateau: iterations without counting after a decrease */
    double min_lr;      /* plateau: lower bound on lr                             */
    double sched_eps;   /* plateau: decreases smaller than this are skipped       */
    /* optimizer (Sec. 6.3 names Adam, SGD and RMSprop): 0 Adam, 1 SGD with
       momentum beta1 (0 = plain), 2 RMSprop with smoothing beta2, no momentum */
    int32_t optimizer;
} orc_opts_t;

/* One optimizer update of a learnable coordinate x with gradient g and state
 * m (first moment / momentum buffer), s (second moment), written as the
 * optimizers define them (PyTorch conventions: SGD without dampening, the
 * buffer starting at the first gradient; RMSprop not centred, eps outside the
 * root; Adam as in Kingma & Ba with bias corrections bc1 = 1-b1^t, bc2 = 1-b2^t). */
static double orc_opt_update(const orc_opts_t *o, double lr, double bc1, double bc2, double x, double g,
                             double *m, double *s)
{
    if (o->optimizer == 1) {
        *m = o->beta1 * *m + g;
        return x - lr * *m;
    }
    if (o->optimizer == 2) {
        *s = o->beta2 * *s + (1.0 - o->beta2) * (g * g);
        return x - lr * (g / (sqrt(*s) + o->eps));
    }
    *m = o->beta1 * *m + (1.0 - o->beta1) * g;
    *s = o->beta2 * *s + (1.0 - o->beta2) * (g * g);
    double mhat = *m / bc1, shat = *s / bc2;
    return x - lr * mhat / (sqrt(shat) + o->eps);
}

/*
 * One DPF solve for one case (Algorithm 1 with Adam).  Iteration k:
 *   1. forward pass: S_calc, residuals, loss L_k and mu_k = max-abs residual;
 *   2. stop test (reading of the loop's `loss < tol`): if mu_k < tol the case
 *      is converged and the voltages just tested are returned; iters = k, the
 *      number of updates applied.  Non-finite mu stops the case (status 2);
 *      reaching k == max_iter stops it unconverged (status 1);
 *   3. gradient (2/m) J_f^T f;
 *   4. optimizer step t = k+1 on the learnable entries (orc_opt_update), by
 *      default Adam (Kingma & Ba):
 *        m <- b1 m + (1-b1) g;  s <- b2 s + (1-b2) g^2;
 *        mhat = m/(1-b1^t);     shat = s/(1-b2^t);
 *        x <- x - lr * mhat / (sqrt(shat) + eps);
 *   5. scheduler step (Algorithm 1 calls it after every optimizer step) with
 *      the loss L_k of this iteration as the plateau metric.
 * vm, va: in = start point, out = returned voltages.
 * state (nullable): [4][n] = m_vm, m_va, s_vm, s_va in/out, t0: in/out step.
 * Returns status 0 converged, 1 max_iter, 2 non-finite.
 */
int32_t orc_solve_adam(int32_t n, const int32_t *rp, const int32_t *ci,
                       const double complex *yv, const int8_t *bus_type,
                       const double complex *s_spec, double *vm, double *va,
                       const orc_opts_t *o, double *state, int32_t *t0,
                       int32_t *iters, double *mu_out, double *lr_out)
{
    double *g_vm = (double *)calloc((size_t)n, sizeof(double));
    double *g_va = (double *)calloc((size_t)n, sizeof(double));
    double *own = NULL;
    if (!state) own = state = (double *)calloc((size_t)(4 * n), sizeof(double));
    double *m_vm = state, *m_va = state + n, *s_vm = state + 2 * n, *s_va = state + 3 * n;
    int32_t tstart = t0 ? *t0 : 0;
    double lr = o->lr, best = INFINITY;
    int32_t bad = 0, cool = 0;
    int32_t status = 1, k = 0;
    double mu = NAN;
    for (k = 0;; ++k) {
        double loss = orc_loss_grad(n, rp, ci, yv, bus_type, vm, va, s_spec, g_vm, g_va, &mu);
        if (!isfinite(mu) || !isfinite(loss)) { status = 2; break; }
        if (mu < o->tol) { status = 0; break; }
        if (k >= o->max_iter) { status = 1; break; }
        double t = (double)(tstart + k + 1);
        double bc1 = 1.0 - pow(o->beta1, t);
        double bc2 = 1.0 - pow(o->beta2, t);
        for (int32_t i = 0; i < n; ++i) {
            if (bus_type[i] == BUS_PQ)
                vm[i] = orc_opt_update(o, lr, bc1, bc2, vm[i], g_vm[i], &m_vm[i], &s_vm[i]);
            if (bus_type[i] != BUS_SLACK)
                va[i] = orc_opt_update(o, lr, bc1, bc2, va[i], g_va[i], &m_va[i], &s_va[i]);
        }
        if (o->sched == 1) {
            /* reduce-on-plateau, mode "min", relative threshold */
            if (loss < best * (1.0 - o->threshold)) { best = loss; bad = 0; }
            else bad += 1;
            if (cool > 0) { cool -= 1; bad = 0; }
            if (bad > o->patience) {
                double nl = lr * o->factor;
                if (nl < o->min_lr) nl = o->min_lr;
                if (lr - nl > o->sched_eps) lr = nl;
                cool = o->cooldown;
                bad = 0;
            }
        } else if (o->sched == 2) {
            /* StepLR: lr = lr0 * gamma^floor(t / step_size), t the persistent count
               of optimizer steps (a resumed solve continues the decay phase) */
            int32_t steps = tstart + k + 1;
            if (o->patience > 0 && steps % o->patience == 0) lr = lr * o->factor;
        }
    }
    if (t0) *t0 = tstart + k;
    *iters = k;
    *mu_out = mu;
    if (lr_out) *lr_out = lr;
    free(g_vm);
    free(g_va);
    free(own);
    return status;
}

/*
 * B independent cases on one shared Y (Sec. 4.2 batches cases; each case here
 * keeps its own Adam state, step count and stop test, which makes the batch
 * equal to B single solves).  Per-case arrays are case-major: x[c*n + i].
 * Cases run in parallel over OpenMP threads; results do not depend on the
 * thread count.
 */
void orc_solve_adam_batch(int32_t B, int32_t n, const int32_t *rp, const int32_t *ci,
                          const double complex *yv, const int8_t *bus_type,
                          const double complex *s_spec, int32_t s_shared,
                          double *vm, double *va, const orc_opts_t *o,
                          int32_t *status, int32_t *iters, double *mu, double *lr_out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < B; ++c) {
        const double complex *s = s_shared ? s_spec : s_spec + (size_t)c * n;
        status[c] = orc_solve_adam(n, rp, ci, yv, bus_type, s, vm + (size_t)c * n,
                                   va + (size_t)c * n, o, NULL, NULL, &iters[c], &mu[c],
                                   lr_out ? &lr_out[c] : NULL);
    }
}

/* Threads the batch solve would use (for reporting). */
int32_t orc_num_threads(void)
{
    int32_t nt = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        nt = (int32_t)omp_get_num_threads();
    }
#endif
    return nt;
}
