/* Drives every entry point of the FP64 oracle (test infrastructure) on small random inputs, for the sanitizer
 * builds of tests/test_sanitizers.py: Gauss-Legendre and Gauss-Lobatto nodes, D, face vectors, contractions,
 * preset matrices, V_d, and the predictor for every physics (generic with A and point sources, per node and
 * per element), on several threads. Exit status 0 when every call returned 0. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int N, m, physics, has_A, coef_per_element, has_src;
    long nelem;
    const double *Q, *params, *A, *B, *src, *dt, *h;
    double *qavg, *favg, *qface, *fface, *favg_fig5;
    int nthreads, nodes;
} oracle_args;

int oracle_gl_nodes(int n, double* xi, double* w);
int oracle_gll_nodes(int n, double* xi, double* w);
int oracle_lagrange_at(int n, const double* xi, double x, double* l);
int oracle_dmatrix(int n, const double* xi, double* D);
int oracle_contract(int n, int m, const double* M, int axis, const double* u, double* out);
int oracle_preset_B(int physics, int m, const double* par, double* B3);
int oracle_apply_Vd(int N, int m, double h, int d, const double* A3, const double* B3, const double* u, double* out);
int oracle_stp(const oracle_args* a);

static unsigned long long state = 88172645463325252ull;
static double rnd(void)  /* xorshift64, uniform in [-1, 1) */
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * 0x1.0p-52 - 1.0;
}
static double* filled(size_t n, double lo, double hi)
{
    double* p = malloc(sizeof(double) * (n ? n : 1));
    for (size_t i = 0; i < n; ++i) p[i] = lo + (hi - lo) * 0.5 * (rnd() + 1.0);
    return p;
}

static int fails = 0;
#define CHECK(call) do { if ((call) != 0) { fprintf(stderr, "failed: %s\n", #call); ++fails; } } while (0)

static void run_stp(int N, int m, int physics, int has_A, int per_elem, int has_src, int nodes)
{
    const long E = 3;
    const int n = N + 1, n3 = n * n * n, n2 = n * n;
    const int np = physics == 0 ? 2 : (physics == 1 ? 3 : (physics == 3 ? 12 : 0));
    oracle_args a;
    memset(&a, 0, sizeof a);
    a.N = N; a.m = m; a.physics = physics; a.has_A = has_A; a.coef_per_element = per_elem; a.has_src = has_src;
    a.nelem = E; a.nthreads = 2; a.nodes = nodes;
    double* Q = filled((size_t)E * n3 * m, -1, 1);
    double* par = NULL;
    double *A = NULL, *B = NULL;
    if (physics == 2) {
        const size_t per = per_elem ? 3 * (size_t)m * m : 3 * (size_t)n3 * m * m;
        B = filled(E * per, -0.3, 0.3);
        if (has_A) A = filled(E * per, -0.3, 0.3);
    } else {
        const size_t per = per_elem ? (size_t)np : (size_t)n3 * np;
        par = filled(E * per, 1.0, 2.0);  /* positive material, metric near the identity below */
        if (physics == 3)
            for (size_t k = 0; k < E * per; k += np)
                for (int j = 0; j < 9; ++j) par[k + 3 + j] = (j % 4 == 0 ? 1.0 : 0.1 * rnd());
    }
    double* src = has_src ? filled((size_t)E * (n3 + m + N), -1, 1) : NULL;
    double dt[3] = {0.01, 0.02, 0.0}, h[3] = {1.0, 0.5, 2.0};
    double* qavg = malloc(sizeof(double) * E * n3 * m);
    double* favg = malloc(sizeof(double) * E * 3 * n3 * m);
    double* fig5 = malloc(sizeof(double) * E * 3 * n3 * m);
    double* qface = malloc(sizeof(double) * E * 6 * n2 * m);
    double* fface = has_A ? malloc(sizeof(double) * E * 6 * n2 * m) : NULL;
    a.Q = Q; a.params = par; a.A = A; a.B = B; a.src = src; a.dt = dt; a.h = h;
    a.qavg = qavg; a.favg = favg; a.qface = qface; a.fface = fface; a.favg_fig5 = fig5;
    CHECK(oracle_stp(&a));
    free(Q); free(par); free(A); free(B); free(src); free(qavg); free(favg); free(fig5); free(qface); free(fface);
}

int main(void)
{
    double xi[16], w[16], D[256], l[16];
    for (int n = 1; n <= 12; ++n) {
        CHECK(oracle_gl_nodes(n, xi, w));
        CHECK(oracle_dmatrix(n, xi, D));
        CHECK(oracle_lagrange_at(n, xi, 0.0, l));
        CHECK(oracle_lagrange_at(n, xi, 1.0, l));
        if (n >= 2) CHECK(oracle_gll_nodes(n, xi, w));
    }
    for (int n = 2; n <= 6; ++n) {
        const int m = 3, n3 = n * n * n;
        CHECK(oracle_gl_nodes(n, xi, w));
        CHECK(oracle_dmatrix(n, xi, D));
        double* u = filled((size_t)n3 * m, -1, 1);
        double* out = malloc(sizeof(double) * n3 * m);
        for (int axis = 0; axis < 3; ++axis) CHECK(oracle_contract(n, m, D, axis, u, out));
        free(u); free(out);
    }
    {
        double par[12] = {2.5, 2.0, 1.5, 1, 0, 0, 0, 1, 0, 0, 0, 1}, B3[3 * 81];
        CHECK(oracle_preset_B(0, 4, par, B3));
        CHECK(oracle_preset_B(1, 9, par, B3));
        CHECK(oracle_preset_B(3, 9, par, B3));
    }
    for (int N = 0; N <= 3; ++N) {
        const int m = 4, n3 = (N + 1) * (N + 1) * (N + 1);
        double* A3 = filled((size_t)3 * n3 * m * m, -1, 1);
        double* B3 = filled((size_t)3 * n3 * m * m, -1, 1);
        double* u = filled((size_t)n3 * m, -1, 1);
        double* out = malloc(sizeof(double) * n3 * m);
        for (int d = 0; d < 3; ++d) CHECK(oracle_apply_Vd(N, m, 0.5, d, A3, B3, u, out));
        free(A3); free(B3); free(u); free(out);
    }
    for (int nodes = 0; nodes <= 1; ++nodes) {
        run_stp(2, 4, 0, 0, 0, 0, nodes);
        run_stp(3, 4, 0, 0, 1, 0, nodes);
        run_stp(2, 9, 1, 0, 0, 0, nodes);
        run_stp(4, 9, 1, 0, 1, 0, nodes);
        run_stp(3, 9, 3, 0, 0, 0, nodes);
        run_stp(2, 9, 3, 0, 1, 0, nodes);
        run_stp(3, 5, 2, 1, 0, 1, nodes);
        run_stp(2, 7, 2, 0, 1, 1, nodes);
        run_stp(1, 1, 2, 1, 0, 0, nodes);
    }
    run_stp(9, 9, 1, 0, 0, 0, 0);
    printf("oracle driver: %d failures\n", fails);
    return fails != 0;
}
