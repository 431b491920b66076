/* Runs every routine of the FP64 oracle (oracle/oracle.c) on small seeded problems, including
 * the degenerate ones (n = 1, d = 1, k = 0, a zero column, q >= 0, a warm start, a trace), so that
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer checks their memory accesses and
 * arithmetic.  Exit status 0 when every result is sane; the sanitizers abort on any finding. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_gram(int64_t d, int64_t n, int64_t k, const double* A, const double* B, double* H,
                 double* h, int nthreads);
void oracle_rescale(int64_t n, int64_t k, const double* H, const double* h, double* s, double* Q,
                    double* q);
int oracle_nqp(int64_t n, const double* Q, const double* q, const double* y0, double tol,
               int64_t max_iter, double* y, int64_t* iters, double* kkt, double* trace);
void oracle_nnls(int64_t d, int64_t n, int64_t k, const double* A, const double* B,
                 const double* Y0, double tol, int64_t max_iter, double* X, int64_t* iters,
                 double* kkt, int32_t* status, double* Q_out, double* q_out, double* s_out,
                 int nthreads);
void oracle_kkt_x(int64_t d, int64_t n, int64_t k, const double* A, const double* B,
                  const double* X, double* r_out, double* F_out, int nthreads);
int oracle_num_threads(void);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static double uniform(void) /* xorshift64*, [0, 1) */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0);
}

static double* vec(int64_t m)
{
    double* p = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    if (!p) exit(3);
    return p;
}

static int failures = 0;

static void expect(int ok, const char* what, int64_t d, int64_t n, int64_t k)
{
    if (!ok) {
        fprintf(stderr, "FAIL %s (d=%lld n=%lld k=%lld)\n", what, (long long)d, (long long)n,
                (long long)k);
        ++failures;
    }
}

/* zero_col >= 0 zeroes that column of A; sign < 0 makes B = -A x (q >= 0, solution 0) */
static void run_case(int64_t d, int64_t n, int64_t k, int zero_col, int sign, int nthreads)
{
    double* A = vec(d * n);
    double* B = vec(d * k);
    double* X = vec(n * k);
    double* Y0 = vec(n * k);
    double* Xs = vec(n * k);
    for (int64_t i = 0; i < d * n; ++i) A[i] = uniform();
    if (zero_col >= 0 && zero_col < n)
        for (int64_t r = 0; r < d; ++r) A[r * n + zero_col] = 0.0;
    for (int64_t i = 0; i < n * k; ++i) Xs[i] = uniform() < 0.4 ? 0.0 : uniform();
    for (int64_t r = 0; r < d; ++r)
        for (int64_t c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i) acc += A[r * n + i] * Xs[i * k + c];
            B[r * k + c] = sign * acc + 0.01 * (uniform() - 0.5);
        }
    for (int64_t i = 0; i < n * k; ++i) Y0[i] = uniform();

    /* the pieces one by one */
    double* H = vec(n * n);
    double* h = vec(n * k);
    double* Q = vec(n * n);
    double* q = vec(n * k);
    double* s = vec(n);
    oracle_gram(d, n, k, A, k > 0 ? B : NULL, H, k > 0 ? h : NULL, nthreads);
    oracle_rescale(n, k, H, h, s, Q, q);
    for (int64_t i = 0; i < n; ++i) expect(s[i] > 0.0 && isfinite(s[i]), "scale", d, n, k);
    if (k > 0) {
        double* qc = vec(n);
        double* y = vec(n);
        double* tr = vec(5 * n + 1);
        int64_t it = -1;
        double kkt = -1.0;
        for (int64_t i = 0; i < n; ++i) qc[i] = q[i * k];
        for (int pass = 0; pass < 2; ++pass) {
            const int st = oracle_nqp(n, Q, qc, pass ? Y0 : NULL, 1e-10, 5 * n, y, &it, &kkt,
                                      pass ? NULL : tr);
            expect(st >= 0 && st <= 3, "nqp status", d, n, k);
            expect(it >= 0 && it <= 5 * n, "nqp iterations", d, n, k);
            expect(isfinite(kkt) && kkt >= 0.0, "nqp residual", d, n, k);
            for (int64_t i = 0; i < n; ++i) expect(y[i] >= 0.0, "nqp y >= 0", d, n, k);
        }
        free(qc);
        free(y);
        free(tr);
    }

    /* end to end, cold and warm, with and without the rescaled problem returned */
    if (k > 0) {
        int64_t* iters = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
        int32_t* status = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
        double* kkt = vec(k);
        double* r = vec(k);
        double* F = vec(k);
        if (!iters || !status) exit(3);
        for (int warm = 0; warm < 2; ++warm) {
            oracle_nnls(d, n, k, A, B, warm ? Y0 : NULL, 1e-9, 5 * n, X, iters, kkt, status,
                        warm ? Q : NULL, warm ? q : NULL, warm ? s : NULL, nthreads);
            for (int64_t c = 0; c < k; ++c) {
                expect(status[c] >= 0 && status[c] <= 3, "nnls status", d, n, k);
                expect(isfinite(kkt[c]), "nnls residual", d, n, k);
            }
            for (int64_t i = 0; i < n * k; ++i) expect(X[i] >= 0.0, "nnls x >= 0", d, n, k);
            oracle_kkt_x(d, n, k, A, B, X, r, F, nthreads);
            for (int64_t c = 0; c < k; ++c)
                expect(isfinite(r[c]) && r[c] >= 0.0 && isfinite(F[c]) && F[c] >= 0.0, "kkt_x",
                       d, n, k);
            if (sign < 0)
                for (int64_t i = 0; i < n * k; ++i) expect(X[i] < 1e-6, "q >= 0 gives x = 0", d, n, k);
        }
        free(iters);
        free(status);
        free(kkt);
        free(r);
        free(F);
    }
    free(A);
    free(B);
    free(X);
    free(Y0);
    free(Xs);
    free(H);
    free(h);
    free(Q);
    free(q);
    free(s);
}

int main(void)
{
    expect(oracle_num_threads() >= 1, "threads", 0, 0, 0);
    run_case(1, 1, 1, -1, 1, 1);
    run_case(5, 1, 3, -1, 1, 2);
    run_case(1, 4, 2, -1, 1, 1);
    run_case(40, 17, 3, 5, 1, 2);
    run_case(40, 17, 0, -1, 1, 1);
    run_case(30, 9, 4, -1, -1, 2);
    run_case(64, 33, 5, 0, 1, 4);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: all checks passed\n");
    return 0;
}
