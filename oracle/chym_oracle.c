/*
 * chym_oracle.c -- plain, slow FP64 CPU oracle of the coherent hyperspin
 * machine (CHYM).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header or constant with the
 * HIP library.
 *
 * Every routine follows a passage of Calvanese Strinati & Conti,
 * "Hyperscaling in the coherent hyperspin machine" (arXiv 2308.02329):
 *
 *   hyperspin layout     PO index j = (p-1) D + mu            main text, NLM paragraph
 *   coupling             C = J_N (x) 1_D  acts per component   text after Eq. (1)
 *   nonlocal loss        W = beta 1_N (x) I_D  -> beta S_p     text after Eq. (1)
 *   round-trip map       Y = Q B - b^2 B (W B^2), A' = (1-d) Y Eq. (2) and the text after it
 *   annealing            C_jl -> alpha_{mu,tau} C_jl            text after Fig. 2
 *   hyperspin energy     E_hs = -sum_pq J_pq s_p . s_q          Eq. (3)
 *   Ising energy / GS    E = -sum_pq J_pq sigma_p sigma_q       opening paragraphs, Eq. (3) with D = 1
 *
 * The continuous-time integrator (oracle_ode_run) is the first-order limit
 * of Eq. (2) for small loss per round trip (time t = gamma tau in photon
 * lifetimes, amplitudes rescaled), integrated by forward Euler:
 *
 *   dx_{p,mu}/dt = (r-1) x_{p,mu} + eps alpha_mu(t) sum_q J_pq x_{q,mu}
 *                  - btil x_{p,mu} sum_nu x_{p,nu}^2 - eta x_{p,mu}^3
 *
 * with eps = b J/(b+d), btil = 1, eta = (kappa L)^2 / (2 beta b^2) for the
 * CHYM and (btil, eta) = (0, 1) for the conventional CIM (beta = 0).
 * oracle_map_run is Eq. (2) itself and pins that limit.
 *
 * Arithmetic: IEEE double, synchronous (Jacobi) update, sums over q in
 * ascending order, expressions evaluated left to right as written.  Build
 * with -ffp-contract=off so that no multiply-add is fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_VERSION 1

int oracle_version(void) { return ORACLE_VERSION; }

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Forward-Euler integration of the normalized CHYM equations.
 *
 *   J      [n][n]        couplings (row p, column q)
 *   pump   [r]           normalized pump r_i = h / h_th per replica
 *   x      [n][r][d]     amplitudes, in/out (row p, replica i, component mu)
 *   alpha  [.][d]        annealing table; step k (global index) uses row k
 *   steps, start_step    integrate steps k = start_step .. start_step+steps-1
 *
 * Replicas never interact, so each replica is integrated on its own; the
 * arithmetic is that of the synchronous update of all of them.
 */
int oracle_ode_run(int n, int d, int r, const double *J, const double *pump,
                   double *x, double eps, double btil, double eta, double dt,
                   int steps, int start_step, const double *alpha, int nthreads) {
    if (n < 0 || d < 1 || r < 0 || steps < 0 || start_step < 0) return -1;
    if (n == 0 || r == 0 || steps == 0) return 0;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int i = 0; i < r; ++i) {
        double *cur = (double *)malloc(sizeof(double) * (size_t)n * d);
        double *nxt = (double *)malloc(sizeof(double) * (size_t)n * d);
        if (!cur || !nxt) { free(cur); free(nxt); bad = 1; continue; }
        for (int p = 0; p < n; ++p)
            for (int mu = 0; mu < d; ++mu)
                cur[p * d + mu] = x[((size_t)p * r + i) * d + mu];
        const double rm1 = pump[i] - 1.0;
        for (int k = 0; k < steps; ++k) {
            const double *al = alpha + (size_t)(start_step + k) * d;
            for (int p = 0; p < n; ++p) {
                double S = 0.0;
                for (int nu = 0; nu < d; ++nu) S = S + cur[p * d + nu] * cur[p * d + nu];
                for (int mu = 0; mu < d; ++mu) {
                    double G = 0.0;
                    for (int q = 0; q < n; ++q) G = G + J[(size_t)p * n + q] * cur[q * d + mu];
                    const double xv = cur[p * d + mu];
                    const double F = rm1 * xv + eps * al[mu] * G - btil * xv * S - eta * xv * xv * xv;
                    nxt[p * d + mu] = xv + dt * F;
                }
            }
            double *t = cur; cur = nxt; nxt = t;
        }
        for (int p = 0; p < n; ++p)
            for (int mu = 0; mu < d; ++mu)
                x[((size_t)p * r + i) * d + mu] = cur[p * d + mu];
        free(cur);
        free(nxt);
    }
    return bad ? -2 : 0;
}

/*
 * Parametric gain of the chi(2) medium, B = K A.  The paper leaves K to its
 * supplement; this is the exact solution of the degenerate, phase-matched
 * coupled-mode equations ds/dz = kappa p s, dp/dz = -kappa s^2 over the
 * length L with p(0) = h, s(0) = A (s^2 + p^2 conserved):
 *   K = P / (P cosh(kL P) - h sinh(kL P)),  P = sqrt(h^2 + A^2).
 * Its small-signal value is exp(kL h) and it is positive for every A.
 */
double oracle_nlm_gain(double a, double h, double kl) {
    const double P = sqrt(h * h + a * a);
    return P / (P * cosh(kl * P) - h * sinh(kl * P));
}

/*
 * The round-trip map of Eq. (2), iterated literally:
 *   B_j   = K(A_j) A_j
 *   Y_j   = (1-b) B_j + b alpha_{mu,tau} sum_l (J_N)_{pl} B_{l,mu}
 *           - beta b^2 B_j sum_nu B_{p,nu}^2
 *   A'_j  = (1 - dd) Y_j
 * J holds the coupling values themselves (+-J, not +-1).  h is per replica.
 */
int oracle_map_run(int n, int d, int r, const double *J, const double *h,
                   double *A, double b, double dd, double kl, double beta,
                   int steps, int start_step, const double *alpha, int nthreads) {
    if (n < 0 || d < 1 || r < 0 || steps < 0 || start_step < 0) return -1;
    if (n == 0 || r == 0 || steps == 0) return 0;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int i = 0; i < r; ++i) {
        double *a = (double *)malloc(sizeof(double) * (size_t)n * d);
        double *bb = (double *)malloc(sizeof(double) * (size_t)n * d);
        if (!a || !bb) { free(a); free(bb); bad = 1; continue; }
        for (int p = 0; p < n; ++p)
            for (int mu = 0; mu < d; ++mu)
                a[p * d + mu] = A[((size_t)p * r + i) * d + mu];
        for (int k = 0; k < steps; ++k) {
            const double *al = alpha + (size_t)(start_step + k) * d;
            for (int j = 0; j < n * d; ++j) bb[j] = oracle_nlm_gain(a[j], h[i], kl) * a[j];
            for (int p = 0; p < n; ++p) {
                double S = 0.0;
                for (int nu = 0; nu < d; ++nu) S = S + bb[p * d + nu] * bb[p * d + nu];
                for (int mu = 0; mu < d; ++mu) {
                    double CB = 0.0;
                    for (int q = 0; q < n; ++q) CB = CB + J[(size_t)p * n + q] * bb[q * d + mu];
                    const double B = bb[p * d + mu];
                    const double Y = (1.0 - b) * B + b * al[mu] * CB - beta * b * b * B * S;
                    a[p * d + mu] = (1.0 - dd) * Y;
                }
            }
        }
        for (int p = 0; p < n; ++p)
            for (int mu = 0; mu < d; ++mu)
                A[((size_t)p * r + i) * d + mu] = a[p * d + mu];
        free(a);
        free(bb);
    }
    return bad ? -2 : 0;
}

/* Ising readout: sigma_p = +1 if the first component x_{p,1} >= 0, else -1
 * (so -0 reads +1 and NaN reads -1).  sigma is [r][n]. */
void oracle_readout(int n, int r, int d, const double *x, int8_t *sigma) {
    for (int i = 0; i < r; ++i)
        for (int p = 0; p < n; ++p)
            sigma[(size_t)i * n + p] = (x[((size_t)p * r + i) * d] >= 0.0) ? 1 : -1;
}

/* Ising energy E = -sum_{p,q} J_pq sigma_p sigma_q (full double sum). */
void oracle_ising_energy(int n, int r, const double *J, const int8_t *sigma, double *E) {
    for (int i = 0; i < r; ++i) {
        const int8_t *s = sigma + (size_t)i * n;
        double e = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q)
                e = e + J[(size_t)p * n + q] * (double)s[p] * (double)s[q];
        E[i] = -e;
    }
}

/* Hyperspin energy of Eq. (3) with unit vectors u_p = x_p / |x_p|
 * (u_p = 0 when x_p = 0). */
void oracle_hs_energy(int n, int r, int d, const double *J, const double *x, double *E) {
    double *u = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * d);
    for (int i = 0; i < r; ++i) {
        for (int p = 0; p < n; ++p) {
            double s = 0.0;
            for (int mu = 0; mu < d; ++mu) {
                const double v = x[((size_t)p * r + i) * d + mu];
                s = s + v * v;
            }
            const double nrm = sqrt(s);
            for (int mu = 0; mu < d; ++mu)
                u[p * d + mu] = (nrm > 0.0) ? x[((size_t)p * r + i) * d + mu] / nrm : 0.0;
        }
        double e = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                double dot = 0.0;
                for (int mu = 0; mu < d; ++mu) dot = dot + u[p * d + mu] * u[q * d + mu];
                e = e + J[(size_t)p * n + q] * dot;
            }
        E[i] = -e;
    }
    free(u);
}

/* Largest share of the extra components in any hyperspin of the replica:
 * max_p sum_{mu>=2} x^2 / |x_p|^2 (0 for a zero hyperspin). */
void oracle_extra_frac(int n, int r, int d, const double *x, double *f) {
    for (int i = 0; i < r; ++i) {
        double m = 0.0;
        for (int p = 0; p < n; ++p) {
            double tot = 0.0, ext = 0.0;
            for (int mu = 0; mu < d; ++mu) {
                const double v = x[((size_t)p * r + i) * d + mu];
                tot = tot + v * v;
                if (mu > 0) ext = ext + v * v;
            }
            if (tot > 0.0 && ext / tot > m) m = ext / tot;
        }
        f[i] = m;
    }
}

/* A run has diverged if any amplitude of its final state is not finite or
 * exceeds 1e3 in magnitude. */
void oracle_diverged(int n, int r, int d, const double *x, uint8_t *flag) {
    for (int i = 0; i < r; ++i) {
        uint8_t bad = 0;
        for (int p = 0; p < n; ++p)
            for (int mu = 0; mu < d; ++mu) {
                const double v = x[((size_t)p * r + i) * d + mu];
                if (!isfinite(v) || fabs(v) > 1e3) bad = 1;
            }
        flag[i] = bad;
    }
}

/*
 * Exact Ising ground state by exhaustive search in Gray-code order.  The
 * last spin is fixed to +1 (E is even in sigma).  Flipping spin k changes
 * E by 4 sigma_k h_k with the local field h_k = sum_q J_kq sigma_q (J_kk = 0
 * is required).  Returns E_GS; best receives one minimizer.
 */
double oracle_bruteforce_gs(int n, const double *J, int8_t *best) {
    if (n <= 0) return 0.0;
    if (n == 1) { if (best) best[0] = 1; return -J[0]; }
    int8_t *s = (int8_t *)malloc((size_t)n);
    double *hf = (double *)malloc(sizeof(double) * (size_t)n);
    for (int p = 0; p < n; ++p) s[p] = 1;
    for (int p = 0; p < n; ++p) {
        double a = 0.0;
        for (int q = 0; q < n; ++q) a = a + J[(size_t)p * n + q] * s[q];
        hf[p] = a;
    }
    double e = 0.0;
    for (int p = 0; p < n; ++p) e = e + s[p] * hf[p];
    e = -e;
    double emin = e;
    if (best) memcpy(best, s, (size_t)n);
    const uint64_t total = (uint64_t)1 << (n - 1);
    for (uint64_t g = 1; g < total; ++g) {
        int k = __builtin_ctzll(g); /* spin flipped between Gray codes g-1 and g */
        e = e + 4.0 * s[k] * hf[k];
        const double two_s = 2.0 * s[k];
        s[k] = (int8_t)-s[k];
        for (int q = 0; q < n; ++q) hf[q] = hf[q] - J[(size_t)q * n + k] * two_s;
        if (e < emin) {
            emin = e;
            if (best) memcpy(best, s, (size_t)n);
        }
    }
    free(s);
    free(hf);
    return emin;
}

/* ---- putative ground state for larger N: single-spin-flip simulated
 * annealing with restarts (the paper quotes "a Monte-Carlo algorithm").
 * Its randomness is xoshiro256** seeded through splitmix64, both as
 * published by Blackman and Vigna. */
static uint64_t sm64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t rotl(uint64_t v, int k) { return (v << k) | (v >> (64 - k)); }
static uint64_t xo_next(uint64_t st[4]) {
    const uint64_t res = rotl(st[1] * 5, 7) * 9;
    const uint64_t t = st[1] << 17;
    st[2] ^= st[0];
    st[3] ^= st[1];
    st[1] ^= st[2];
    st[0] ^= st[3];
    st[2] ^= t;
    st[3] = rotl(st[3], 45);
    return res;
}
static double xo_unif(uint64_t st[4]) { return (double)(xo_next(st) >> 11) * 0x1.0p-53; }

double oracle_anneal_gs(int n, const double *J, int sweeps, int restarts, uint64_t seed,
                        double t_hot, double t_cold, int8_t *best, int nthreads) {
    if (n <= 0) return 0.0;
    set_threads(nthreads);
    double gbest = INFINITY;
    int8_t *gsig = (int8_t *)malloc((size_t)n);
#pragma omp parallel
    {
        int8_t *s = (int8_t *)malloc((size_t)n);
        double *hf = (double *)malloc(sizeof(double) * (size_t)n);
        double lbest = INFINITY;
        int8_t *lsig = (int8_t *)malloc((size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int rs = 0; rs < restarts; ++rs) {
            uint64_t sd = seed ^ ((uint64_t)rs * 0xD1B54A32D192ED03ull);
            uint64_t st[4] = {sm64(&sd), sm64(&sd), sm64(&sd), sm64(&sd)};
            for (int p = 0; p < n; ++p) s[p] = (xo_next(st) >> 63) ? 1 : -1;
            for (int p = 0; p < n; ++p) {
                double a = 0.0;
                for (int q = 0; q < n; ++q) a = a + J[(size_t)p * n + q] * s[q];
                hf[p] = a;
            }
            double e = 0.0;
            for (int p = 0; p < n; ++p) e = e + s[p] * hf[p];
            e = -e;
            double eb = e;
            for (int sw = 0; sw < sweeps; ++sw) {
                const double frac = sweeps > 1 ? (double)sw / (double)(sweeps - 1) : 1.0;
                const double T = t_hot * pow(t_cold / t_hot, frac);
                for (int k = 0; k < n; ++k) {
                    const double de = 4.0 * s[k] * hf[k];
                    if (de <= 0.0 || xo_unif(st) < exp(-de / T)) {
                        const double two_s = 2.0 * s[k];
                        s[k] = (int8_t)-s[k];
                        for (int q = 0; q < n; ++q) hf[q] = hf[q] - J[(size_t)q * n + k] * two_s;
                        e = e + de;
                        if (e < eb) eb = e;
                        if (e < lbest) { lbest = e; memcpy(lsig, s, (size_t)n); }
                    }
                }
            }
            if (e < lbest) { lbest = e; memcpy(lsig, s, (size_t)n); }
            (void)eb;
        }
#pragma omp critical
        {
            if (lbest < gbest) { gbest = lbest; memcpy(gsig, lsig, (size_t)n); }
        }
        free(s);
        free(hf);
        free(lsig);
    }
    if (best) memcpy(best, gsig, (size_t)n);
    free(gsig);
    return gbest;
}
