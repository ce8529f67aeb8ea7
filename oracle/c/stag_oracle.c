/*
 * Plain C + OpenMP fp64 oracle for the staggered normal operator and CG.
 *
 * TEST INFRASTRUCTURE: loaded only by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark. It is deliberately untuned: one loop
 * iteration per output site, complex arithmetic from <complex.h>, no
 * blocking or vectorisation beyond what the compiler does by itself.
 *
 * What it computes (Jang, Kim and Lee, Lattice 2011):
 *   Eq.5  (D chi)(x) = sum_mu eta_mu(x) U_mu(x) chi(x+mu)
 *                             - eta_mu(x-mu) U_mu(x-mu)^+ chi(x-mu)
 *         with eta_mu(x) = (-1)^(x_0+...+x_{mu-1}) multiplied into the links
 *         (Sec.2), periodic boundaries;
 *   Eq.3  A = -D^2 + m^2 on the even sites, i.e. A chi = m^2 chi - D_eo D_oe chi;
 *   the improved operator: Eq.5 over fat links plus the three-hop terms
 *         eta_mu(x) N_mu(x) chi(x+3mu) - eta_mu(x-3mu) N_mu(x-3mu)^+ chi(x-3mu)
 *         over caller-supplied long links N;
 *   Fig.1 conjugate gradient in fp64, stopping on |r| <= tol |b|, then a
 *         true-residual check that restarts from r = b - A x if it fails.
 *
 * Layouts: links complex128 [t][z][y][x][mu][a][b]; parity-p vectors
 * complex128 [s][c] with s = lex / 2 over the sites of that parity.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    int L[4];
    long V, Vh;
} lat_t;

static int lat_init(lat_t* lt, const int* L) {
    for (int mu = 0; mu < 4; ++mu) {
        if (L[mu] < 2 || (L[mu] & 1)) return -1;
        lt->L[mu] = L[mu];
    }
    lt->V = (long)L[0] * L[1] * L[2] * L[3];
    lt->Vh = lt->V / 2;
    return 0;
}

static long lex_of(const lat_t* lt, const int c[4]) {
    return c[0] + (long)lt->L[0] * (c[1] + (long)lt->L[1] * (c[2] + (long)lt->L[2] * c[3]));
}

/* coordinates of the site with checkerboard index s on parity p */
static void coords_of(const lat_t* lt, long s, int p, int c[4]) {
    long hx = lt->L[0] / 2;
    long row = s / hx;
    int xh = (int)(s % hx);
    c[1] = (int)(row % lt->L[1]);
    row /= lt->L[1];
    c[2] = (int)(row % lt->L[2]);
    c[3] = (int)(row / lt->L[2]);
    c[0] = 2 * xh + ((c[1] + c[2] + c[3] + p) & 1);
}

static double eta_of(int mu, const int c[4]) {
    int s = 0;
    for (int nu = 0; nu < mu; ++nu) s += c[nu];
    return (s & 1) ? -1.0 : 1.0;
}

static const cplx* link_at(const cplx* U, long lex, int mu) { return U + (lex * 4 + mu) * 9; }

/* acc += eta W(x) in(x + dist mu) - eta W(x - dist mu)^+ in(x - dist mu) */
static void add_hops(const lat_t* lt, const cplx* W, const cplx* in, const int c[4], int mu,
                     int dist, cplx acc[3]) {
    int f[4] = {c[0], c[1], c[2], c[3]};
    int b[4] = {c[0], c[1], c[2], c[3]};
    f[mu] = (f[mu] + dist) % lt->L[mu];
    b[mu] = ((b[mu] - dist) % lt->L[mu] + lt->L[mu]) % lt->L[mu];
    long lf = lex_of(lt, f), lb = lex_of(lt, b);
    const cplx* uf = link_at(W, lex_of(lt, c), mu);
    const cplx* ub = link_at(W, lb, mu);
    const cplx* vf = in + (lf / 2) * 3;
    const cplx* vb = in + (lb / 2) * 3;
    double ef = eta_of(mu, c), eb = eta_of(mu, b);
    for (int a = 0; a < 3; ++a) {
        cplx sf = 0, sb = 0;
        for (int k = 0; k < 3; ++k) {
            sf += uf[a * 3 + k] * vf[k];
            sb += conj(ub[k * 3 + a]) * vb[k];
        }
        acc[a] += ef * sf - eb * sb;
    }
}

/* out (parity 1 - p_in) = D in (parity p_in); N (long links) may be NULL */
static void dslash(const lat_t* lt, const cplx* U, const cplx* N, const cplx* in, cplx* out,
                   int p_in) {
    int p_out = 1 - p_in;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < lt->Vh; ++s) {
        int c[4];
        coords_of(lt, s, p_out, c);
        cplx acc[3] = {0, 0, 0};
        for (int mu = 0; mu < 4; ++mu) {
            add_hops(lt, U, in, c, mu, 1, acc);
            if (N) add_hops(lt, N, in, c, mu, 3, acc);
        }
        for (int a = 0; a < 3; ++a) out[s * 3 + a] = acc[a];
    }
}

static void apply_A(const lat_t* lt, const cplx* U, const cplx* N, double m, const cplx* in,
                    cplx* out, cplx* tmp) {
    dslash(lt, U, N, in, tmp, 0);
    dslash(lt, U, N, tmp, out, 1);
    long n = lt->Vh * 3;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) out[i] = m * m * in[i] - out[i];
}

static double dot_re(const cplx* a, const cplx* b, long n) {
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (long i = 0; i < n; ++i) s += creal(conj(a[i]) * b[i]);
    return s;
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* N: long links of the improved operator, or NULL for Eq.5 */
int oracle_dslash(const int* L, const double* U, const double* N, const double* in, double* out,
                  int p_in) {
    lat_t lt;
    if (lat_init(&lt, L) || (p_in != 0 && p_in != 1)) return -1;
    dslash(&lt, (const cplx*)U, (const cplx*)N, (const cplx*)in, (cplx*)out, p_in);
    return 0;
}

int oracle_apply_A(const int* L, const double* U, const double* N, double m, const double* in,
                   double* out) {
    lat_t lt;
    if (lat_init(&lt, L)) return -1;
    cplx* tmp = malloc(sizeof(cplx) * lt.Vh * 3);
    if (!tmp) return -2;
    apply_A(&lt, (const cplx*)U, (const cplx*)N, m, (const cplx*)in, (cplx*)out, tmp);
    free(tmp);
    return 0;
}

/*
 * Fig.1 CG. x holds the result (x0 = 0). max_iter <= 0 means
 * min(10 n, 10^6). Stats: iters[0] = iterations, true_rel[0] = |b-Ax|/|b|.
 * Returns 0 on convergence, 1 if max_iter was reached, 2 on breakdown,
 * negative on bad arguments or allocation failure.
 */
int oracle_cg(const int* L, const double* U_, double m, const double* b_, double* x_,
              double tol, long max_iter, long* iters, double* true_rel) {
    lat_t lt;
    if (lat_init(&lt, L)) return -1;
    const cplx* U = (const cplx*)U_;
    const cplx* b = (const cplx*)b_;
    cplx* x = (cplx*)x_;
    long n = lt.Vh * 3;
    if (max_iter <= 0) max_iter = (10 * n < 1000000) ? 10 * n : 1000000;
    cplx* r = malloc(sizeof(cplx) * n);
    cplx* d = malloc(sizeof(cplx) * n);
    cplx* q = malloc(sizeof(cplx) * n);
    cplx* tmp = malloc(sizeof(cplx) * n);
    if (!r || !d || !q || !tmp) {
        free(r); free(d); free(q); free(tmp);
        return -2;
    }
    memset(x, 0, sizeof(cplx) * n);
    double bb = dot_re(b, b, n);
    int status = 0;
    long i = 0;
    double true_rr = 0.0;
    if (bb > 0.0) {
        double stop = tol * tol * bb;
        memcpy(r, b, sizeof(cplx) * n); /* r = b - A*0 */
        memcpy(d, r, sizeof(cplx) * n);
        double delta_new = bb;
        for (;;) {
            while (i < max_iter && delta_new > stop) {
                apply_A(&lt, U, NULL, m, d, q, tmp);
                double dq = dot_re(d, q, n);
                if (!(dq > 0.0) || !isfinite(dq)) { status = 2; break; }
                double alpha = delta_new / dq;
#pragma omp parallel for schedule(static)
                for (long k = 0; k < n; ++k) {
                    x[k] += alpha * d[k];
                    r[k] -= alpha * q[k];
                }
                double delta_old = delta_new;
                delta_new = dot_re(r, r, n);
                double beta = delta_new / delta_old;
#pragma omp parallel for schedule(static)
                for (long k = 0; k < n; ++k) d[k] = r[k] + beta * d[k];
                ++i;
            }
            apply_A(&lt, U, NULL, m, x, q, tmp);
#pragma omp parallel for schedule(static)
            for (long k = 0; k < n; ++k) tmp[k] = b[k] - q[k];
            true_rr = dot_re(tmp, tmp, n);
            if (status != 0 || true_rr <= stop || i >= max_iter) break;
            memcpy(r, tmp, sizeof(cplx) * n);
            memcpy(d, r, sizeof(cplx) * n);
            delta_new = true_rr;
        }
        if (status == 0 && true_rr > stop) status = 1;
    }
    if (iters) *iters = i;
    if (true_rel) *true_rel = bb > 0.0 ? sqrt(true_rr / bb) : 0.0;
    free(r); free(d); free(q); free(tmp);
    return status;
}

/* Run exactly n_iter Fig.1 iterations from x = 0 (a bounded timing sample). */
int oracle_cg_fixed(const int* L, const double* U, double m, const double* b, double* x,
                    long n_iter) {
    long it = 0;
    double tr = 0.0;
    int rc = oracle_cg(L, U, m, b, x, 0.0, n_iter, &it, &tr);
    return rc < 0 ? rc : 0;
}
