/*
 * Plain FP64 CPU oracle of the anti-lopsided NNLS method (Nguyen & Ho, arXiv 1502.01645).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no source, header, table or
 * helper with the HIP library; the two only meet through the seeded input generators.
 *
 * Every routine is the paper's definition written out in straightforward loops, in double
 * precision, with no blocking, fusion or reordering beyond what the definition states:
 *
 *   oracle_gram      H = A^T A and h = -A^T B                     (Problem (2), NQP form)
 *   oracle_rescale   Q_ij = H_ij / sqrt(H_ii H_jj), q_i = h_i / sqrt(H_ii)
 *                    (Algorithm 1, second and third steps; rescaling (4)-(5); the special
 *                     case H_ii = 0 keeps x_i = y_i, i.e. a unit scale)
 *   oracle_nqp       Algorithm 2: gradient method with exact line search on the passive set
 *   oracle_nnls      Algorithm 1 end to end, column by column over a block of right-hand sides
 *   oracle_kkt_x     relative KKT residual and objective of an x against the original (A, b)
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *   - the update is x_{k+1} = [x_k - alpha * gbar]_+ (Algorithm 2 uses the minus sign; the
 *     prose of Section 3 prints a plus, which would ascend);
 *   - epsilon is not given: the loop stops when the relative KKT residual
 *         r(y) = || min(y, Qy + q) ||_2 / ||q||_2     (||q|| = 0: unnormalised)
 *     is at most tol, when the passive set is empty, or after max_iter updates;
 *   - the stop test runs at the top of each pass on the current iterate, and the latest
 *     iterate is returned;
 *   - a zero-length column (H_ii = 0) gets scale 1, so its row and column of Q and its q
 *     entry are zero and it never enters the passive set;
 *   - a line-search denominator that is not positive and finite ends the solve with status
 *     BREAKDOWN; a non-finite input or iterate ends it with status NONFINITE.
 *
 * Layouts: all matrices are row-major.  A is [d, n], B is [d, k], H and Q are [n, n],
 * h and q are [n, k], X is [n, k].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_CONVERGED = 0, OR_MAXITER = 1, OR_BREAKDOWN = 2, OR_NONFINITE = 3 };

/* Planted-mistake switch used only by the pin-strength test: the default build (PLANT 0) is the
 * oracle proper; each nonzero value introduces one plausible slip so the test can show that at
 * least one pin catches it. */
#ifndef PLANT
#define PLANT 0
#endif

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* H = A^T A, h = -A^T B (Problem (2)).  H is symmetric: the upper triangle is computed and
 * mirrored.  h may be NULL when k == 0. */
void oracle_gram(int64_t d, int64_t n, int64_t k, const double* A, const double* B,
                 double* H, double* h, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i; j < n; ++j) {
            double acc = 0.0;
            for (int64_t r = 0; r < d; ++r) acc += A[r * n + i] * A[r * n + j];
#if PLANT == 1
            if (i != j) acc *= 0.999; /* planted: perturbed off-diagonal Gram entries */
#endif
            H[i * n + j] = acc;
            H[j * n + i] = acc;
        }
        for (int64_t c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int64_t r = 0; r < d; ++r) acc += A[r * n + i] * B[r * k + c];
#if PLANT == 2
            h[i * k + c] = acc; /* planted: dropped minus sign of h */
#else
            h[i * k + c] = -acc;
#endif
        }
    }
}

/* Scale vector s_i = sqrt(H_ii) (1 where H_ii == 0), Q = H / (s s^T), q = h / s
 * (Algorithm 1; rescaling (4); Problem (5)).  The diagonal of Q is set to exactly 1 where
 * H_ii > 0, as the Remark of Section 3 states (Q_ii = cos(A_i, A_i) = 1). */
void oracle_rescale(int64_t n, int64_t k, const double* H, const double* h, double* s,
                    double* Q, double* q)
{
    for (int64_t i = 0; i < n; ++i) {
        double hii = H[i * n + i];
#if PLANT == 3
        s[i] = hii > 0.0 ? hii : 1.0; /* planted: scale by H_ii instead of sqrt(H_ii) */
#else
        s[i] = hii > 0.0 ? sqrt(hii) : 1.0;
#endif
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) Q[i * n + j] = H[i * n + j] / (s[i] * s[j]);
        if (H[i * n + i] > 0.0) Q[i * n + i] = 1.0;
        for (int64_t c = 0; c < k; ++c) q[i * k + c] = h[i * k + c] / s[i];
    }
}

static int all_finite(int64_t m, const double* v)
{
    for (int64_t i = 0; i < m; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static double norm2(int64_t n, const double* v)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += v[i] * v[i];
    return sqrt(acc);
}

/* || min(y, g) ||_2: zero exactly when y >= 0, g >= 0 and y .* g = 0 (the KKT conditions of
 * the non-negative quadratic program). */
static double kkt_abs(int64_t n, const double* y, const double* g)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double m = y[i] < g[i] ? y[i] : g[i];
        acc += m * m;
    }
    return sqrt(acc);
}

/* out = Q v (dense, Q [n, n]). */
static void matvec(int64_t n, const double* Q, const double* v, double* out)
{
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) acc += Q[i * n + j] * v[j];
        out[i] = acc;
    }
}

/*
 * Algorithm 2 on one right-hand side: minimise f(y) = 1/2 y^T Q y + q^T y subject to y >= 0.
 *
 * y0 may be NULL (the algorithm's start x^0 = 0, gradient = q); otherwise the gradient starts
 * as Q y0 + q.  Each pass: the passive set P = {i : y_i > 0 or grad_i < 0} and the masked
 * gradient gbar (grad on P, 0 elsewhere); the exact step alpha = ||gbar||^2 / gbar^T Q gbar
 * (derivation after Algorithm 2); the projected update y' = [y - alpha gbar]_+; the incremental
 * gradient grad += Q (y' - y), formed as a second product as the algorithm writes it.
 *
 * Outputs: y [n], *iters = number of completed updates, *kkt = relative KKT residual of the
 * returned y with a freshly recomputed gradient, return value = status.
 * trace (may be NULL) receives the running relative residual at the top of every pass.
 */
int oracle_nqp(int64_t n, const double* Q, const double* q, const double* y0, double tol,
               int64_t max_iter, double* y, int64_t* iters, double* kkt, double* trace)
{
    double* g = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 4);
    double* p = g + n;
    double* w = p + n;
    double* dy = w + n;
    int status = OR_MAXITER;
    int64_t it = 0;
    double qn = norm2(n, q);
    double scale = qn > 0.0 ? qn : 1.0;

    if (!all_finite(n * n, Q) || !all_finite(n, q) || (y0 && !all_finite(n, y0))) {
        for (int64_t i = 0; i < n; ++i) y[i] = y0 ? y0[i] : 0.0;
        *iters = 0;
        *kkt = NAN;
        free(g);
        return OR_NONFINITE;
    }
    if (y0) {
        for (int64_t i = 0; i < n; ++i) y[i] = y0[i] > 0.0 ? y0[i] : 0.0;
        matvec(n, Q, y, g);
        for (int64_t i = 0; i < n; ++i) g[i] += q[i];
    } else {
        for (int64_t i = 0; i < n; ++i) {
            y[i] = 0.0;
            g[i] = q[i];
        }
    }

    for (it = 0;; ++it) {
        if (!all_finite(n, g) || !all_finite(n, y)) {
            status = OR_NONFINITE;
            break;
        }
        int64_t npass = 0;
        double num = 0.0;
        for (int64_t i = 0; i < n; ++i) {
#if PLANT == 4
            int passive = (y[i] > 0.0) || (g[i] > 0.0); /* planted: wrong sign in the passive test */
#else
            int passive = (y[i] > 0.0) || (g[i] < 0.0);
#endif
            p[i] = passive ? g[i] : 0.0;
            npass += passive;
            num += p[i] * p[i];
        }
        double r = kkt_abs(n, y, g) / scale;
        if (trace && it < max_iter + 1) trace[it] = r;
        if (npass == 0 || r <= tol) {
            status = OR_CONVERGED;
            break;
        }
        if (it >= max_iter) {
            status = OR_MAXITER;
            break;
        }
        matvec(n, Q, p, w);
        double den = 0.0;
        for (int64_t i = 0; i < n; ++i) den += p[i] * w[i];
        if (!(den > 0.0) || !isfinite(den)) {
            status = OR_BREAKDOWN;
            break;
        }
        double alpha = num / den;
#if PLANT == 5
        alpha = num / (2.0 * den); /* planted: half the exact step */
#endif
        for (int64_t i = 0; i < n; ++i) {
#if PLANT == 6
            double v = y[i] + alpha * p[i]; /* planted: the plus sign of the prose */
#else
            double v = y[i] - alpha * p[i];
#endif
            double ynew = v > 0.0 ? v : 0.0;
            dy[i] = ynew - y[i];
            y[i] = ynew;
        }
        matvec(n, Q, dy, w);
        for (int64_t i = 0; i < n; ++i) g[i] += w[i];
    }

    /* Report the residual with an exact gradient, not the incrementally updated one. */
    matvec(n, Q, y, g);
    for (int64_t i = 0; i < n; ++i) g[i] += q[i];
    *kkt = kkt_abs(n, y, g) / scale;
    *iters = it;
    free(g);
    return status;
}

/*
 * Algorithm 1 over a block of k right-hand sides sharing A: Gram and rescale once, then
 * Algorithm 2 per column, then x = y / s (rescaling (4)).
 *
 * A [d, n], B [d, k], Y0 [n, k] or NULL, X [n, k].  Per column: iters, kkt (relative residual in
 * the rescaled problem), status.  Q_out [n, n], q_out [n, k] and s_out [n] may be NULL; when
 * given they receive the rescaled problem.  Columns run in parallel over nthreads threads.
 */
void oracle_nnls(int64_t d, int64_t n, int64_t k, const double* A, const double* B,
                 const double* Y0, double tol, int64_t max_iter, double* X, int64_t* iters,
                 double* kkt, int32_t* status, double* Q_out, double* q_out, double* s_out,
                 int nthreads)
{
    double* H = (double*)malloc(sizeof(double) * (size_t)(n * n + n * k + n * n + n * k + n) + 8);
    double* h = H + n * n;
    double* Q = h + n * k;
    double* q = Q + n * n;
    double* s = q + n * k;
    oracle_gram(d, n, k, A, B, H, h, nthreads);
    oracle_rescale(n, k, H, h, s, Q, q);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < k; ++c) {
        double* buf = (double*)malloc(sizeof(double) * (size_t)(3 * n + 1));
        double* qc = buf;
        double* yc = qc + n;
        double* y0c = yc + n;
        for (int64_t i = 0; i < n; ++i) {
            qc[i] = q[i * k + c];
            if (Y0) y0c[i] = Y0[i * k + c];
        }
        status[c] = oracle_nqp(n, Q, qc, Y0 ? y0c : NULL, tol, max_iter, yc, &iters[c], &kkt[c],
                               NULL);
        for (int64_t i = 0; i < n; ++i) X[i * k + c] = yc[i] / s[i];
        free(buf);
    }
    if (Q_out) memcpy(Q_out, Q, sizeof(double) * (size_t)(n * n));
    if (q_out) memcpy(q_out, q, sizeof(double) * (size_t)(n * k));
    if (s_out) memcpy(s_out, s, sizeof(double) * (size_t)n);
    free(H);
}

/*
 * Quality of a candidate x against the original data, in the variables of Problem (1):
 *   F(x)  = 1/2 || A x - b ||^2, formed from the residual (never from x^T H x terms);
 *   r(x)  = || min(s .* x, grad F(x) ./ s) ||_2 / || A^T b ./ s ||_2, s_i = ||A_i|| (1 if 0),
 * which equals the rescaled-space residual of y = s .* x.  One column at a time, in parallel.
 * A [d, n], B [d, k], X [n, k]; outputs r[k], F[k].
 */
void oracle_kkt_x(int64_t d, int64_t n, int64_t k, const double* A, const double* B,
                  const double* X, double* r_out, double* F_out, int nthreads)
{
    double* s = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t r = 0; r < d; ++r) acc += A[r * n + i] * A[r * n + i];
        s[i] = acc > 0.0 ? sqrt(acc) : 1.0;
    }
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < k; ++c) {
        double* res = (double*)malloc(sizeof(double) * (size_t)(d + 1));
        double F = 0.0;
        for (int64_t r = 0; r < d; ++r) {
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i) acc += A[r * n + i] * X[i * k + c];
            res[r] = acc - B[r * k + c];
            F += res[r] * res[r];
        }
        double kk = 0.0, qq = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double gr = 0.0, atb = 0.0;
            for (int64_t r = 0; r < d; ++r) {
                gr += A[r * n + i] * res[r];
                atb += A[r * n + i] * B[r * k + c];
            }
            double yi = s[i] * X[i * k + c];
            double gi = gr / s[i];
            double m = yi < gi ? yi : gi;
            kk += m * m;
            qq += (atb / s[i]) * (atb / s[i]);
        }
        r_out[c] = qq > 0.0 ? sqrt(kk) / sqrt(qq) : sqrt(kk);
        F_out[c] = 0.5 * F;
        free(res);
    }
    free(s);
}
