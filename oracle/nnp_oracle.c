/*
 * nnp_oracle.c -- plain FP64 CPU oracle for the gas-phase NNP energy, forces
 * and velocity-Verlet integration.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant with the HIP path; it exists so that the
 * HIP path can be checked against a slow, obviously correct definition.
 *
 * What it computes (paper: the force-provider contract of the Methods
 * section -- a callable returns a potential energy and the engine obtains
 * forces as minus its gradient; the NVE validation of the Results section):
 *
 *   O1  pair sets: P_R(i) = { j != i : r_ij < 5.2 },
 *                  P_A(i) = { j != i : r_ij < 3.5 }    (brute force, O(N^2))
 *   O2  cosine cutoff fc(r; Rc) = cos(pi r / Rc)/2 + 1/2 for r < Rc, else 0
 *   O3  radial features G[16 s_j + k] = sum_j exp(-16 (r - Rk)^2) fc(r; 5.2),
 *       Rk = 0.9 + 0.28 k, k = 0..15
 *   O4  angular features, unordered pairs j < k of P_A(i):
 *       c' = 0.95 cos(theta_ijk),
 *       A_n = (1 + c' cos(t_n) + sqrt(1 - c'^2) sin(t_n))^32,  t_n = (2n+1) pi / 16
 *       B_m = exp(-8 ((r_ij + r_ik)/2 - Q_m)^2),                Q_m = 0.9 + 0.65 m
 *       G[64 + 32 p(s_j, s_k) + 8 m + n] += 2^(1-32) A_n B_m fc(r_ij; 3.5) fc(r_ik; 3.5)
 *       p indexes unordered element pairs HH HC HN HO CC CN CO NN NO OO
 *   O5  per-element network 384 -> 160 -> 128 -> 96 -> 1, CELU(alpha = 0.1)
 *       between layers, linear output; weights [out][in] row-major per element
 *       H, C, N, O: W1 b1 W2 b2 W3 b3 W4 b4 (float32 blob, widened exactly)
 *   O6  E = sum_i E_i
 *   O7  F_a = -dE/dx_a, analytic: network backward to g_i = dE_i/dG_i, then
 *       the chain rule through every pair and triple term (gather form:
 *       each atom sums the derivative of every E_i that depends on it)
 *   O8  velocity Verlet: v += dt/2 kappa F/m; x += dt v; F = F(x);
 *       v += dt/2 kappa F/m; kappa = 9.64853321e-3 A fs^-2 per eV A^-1 amu^-1
 *
 *   O9  Langevin dynamics (the thermostatted runs of the Results section,
 *       friction 0.1 ps^-1), BAOAB splitting (Leimkuhler and Matthews,
 *       J. Chem. Phys. 138, 174102 (2013)), velocities at whole steps:
 *       v += dt/2 kappa F/m; x += dt/2 v;
 *       v = a v + sqrt((1 - a^2) kB T kappa / m) z,   a = exp(-gamma dt);
 *       x += dt/2 v; F = F(x); v += dt/2 kappa F/m
 *   O10 noise z of atom c (caller index) in the step that starts at step
 *       count s: Philox4x64-10 (Salmon et al., SC'11) of the counter
 *       (c, s, 0, 0) under the key (seed, 0); each 64-bit word w gives
 *       u = (floor(w / 2^11) + 1/2) 2^-53, and Box-Muller turns (u0, u1),
 *       (u2, u3) into sqrt(-2 ln u0) (cos, sin)(2 pi u1) and
 *       sqrt(-2 ln u2) cos(2 pi u3): z = those three values for x, y, z
 *
 * Periodic orthorhombic boxes are handled in the Python wrapper by explicit
 * periodic images around the box fed to these gas-phase routines (no minimum
 * image convention), see periodic_energy_forces.
 *
 * The harmonic test model E = sum(x^2) (the paper's Model42 example) and a
 * force-free model are provided as further force models for the integrators.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NSPECIES 4
#define NRAD 16
#define NSHELL 4
#define NSECTOR 8
#define NFEAT 384
#define H1 160
#define H2 128
#define H3 96

static const double PI = 3.14159265358979323846;
static const double RC_RAD = 5.2;
static const double RC_ANG = 3.5;
static const double ETA_RAD = 16.0;
static const double ETA_ANG = 8.0;
static const double ZETA = 32.0;
static const double COS_SCALE = 0.95;
static const double CELU_ALPHA = 0.1;
static const double KAPPA = 9.64853321e-3;
static const double KB = 8.617333262e-5; /* eV / K */

#define PER_ELEMENT (H1 * NFEAT + H1 + H2 * H1 + H2 + H3 * H2 + H3 + H3 + 1)

static double radial_centre(int k) { return 0.9 + 0.28 * k; }
static double shell_centre(int m) { return 0.9 + 0.65 * m; }
static double sector_centre(int n) { return (2.0 * n + 1.0) * PI / 16.0; }

/* O2 */
static double cutoff(double r, double rc) { return r < rc ? 0.5 * cos(PI * r / rc) + 0.5 : 0.0; }
static double cutoff_deriv(double r, double rc) { return r < rc ? -0.5 * PI / rc * sin(PI * r / rc) : 0.0; }

/* index of the unordered element pair {a, b} in HH HC HN HO CC CN CO NN NO OO */
static int pair_type(int a, int b)
{
    static const int table[4][4] = {{0, 1, 2, 3}, {1, 4, 5, 6}, {2, 5, 7, 8}, {3, 6, 8, 9}};
    return table[a][b];
}

/* ------------------------------------------------------------------ O1 --- */

static double dist(const double* pos, int i, int j, double d[3])
{
    d[0] = pos[3 * j + 0] - pos[3 * i + 0];
    d[1] = pos[3 * j + 1] - pos[3 * i + 1];
    d[2] = pos[3 * j + 2] - pos[3 * i + 2];
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* Ordered pairs (i, j), i != j, r_ij < rc, in lexicographic order.  Returns
 * the number of pairs; writes at most cap of them. */
long oracle_pairs(int n, const double* pos, double rc, int* out_i, int* out_j, long cap)
{
    long cnt = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double d[3];
            if (j == i) continue;
            if (dist(pos, i, j, d) < rc) {
                if (cnt < cap) { out_i[cnt] = i; out_j[cnt] = j; }
                ++cnt;
            }
        }
    return cnt;
}

/* Neighbour lists within RC_RAD, ascending index (brute force). */
typedef struct {
    int n;
    int* start; /* n + 1 */
    int* idx;
} nlist;

static void nlist_build(nlist* L, int n, const double* pos)
{
    int* cnt = (int*)calloc((size_t)n, sizeof(int));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double d[3];
            if (j != i && dist(pos, i, j, d) < RC_RAD) cnt[i]++;
        }
    L->n = n;
    L->start = (int*)malloc(sizeof(int) * (size_t)(n + 1));
    L->start[0] = 0;
    for (int i = 0; i < n; ++i) L->start[i + 1] = L->start[i] + cnt[i];
    L->idx = (int*)malloc(sizeof(int) * (size_t)(L->start[n] > 0 ? L->start[n] : 1));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        int w = L->start[i];
        for (int j = 0; j < n; ++j) {
            double d[3];
            if (j != i && dist(pos, i, j, d) < RC_RAD) L->idx[w++] = j;
        }
    }
    free(cnt);
}

static void nlist_free(nlist* L)
{
    free(L->start);
    free(L->idx);
}

/* ---------------------------------------------------------- O3, O4 ------ */

static void descriptor(const double* pos, const int* sp, const nlist* L, int i, double* G)
{
    memset(G, 0, sizeof(double) * NFEAT);
    /* O3 radial */
    for (int t = L->start[i]; t < L->start[i + 1]; ++t) {
        int j = L->idx[t];
        double d[3];
        double r = dist(pos, i, j, d);
        double f = cutoff(r, RC_RAD);
        for (int k = 0; k < NRAD; ++k) {
            double x = r - radial_centre(k);
            G[NRAD * sp[j] + k] += exp(-ETA_RAD * x * x) * f;
        }
    }
    /* O4 angular: unordered pairs j < k of P_A(i) */
    for (int a = L->start[i]; a < L->start[i + 1]; ++a) {
        int j = L->idx[a];
        double dj[3];
        double rj = dist(pos, i, j, dj);
        if (!(rj < RC_ANG)) continue;
        for (int b = a + 1; b < L->start[i + 1]; ++b) {
            int k = L->idx[b];
            double dk[3];
            double rk = dist(pos, i, k, dk);
            if (!(rk < RC_ANG)) continue;
            double c = (dj[0] * dk[0] + dj[1] * dk[1] + dj[2] * dk[2]) / (rj * rk);
            double cp = COS_SCALE * c;
            double sp_ = sqrt(1.0 - cp * cp);
            double w = ldexp(1.0, 1 - (int)ZETA) * cutoff(rj, RC_ANG) * cutoff(rk, RC_ANG);
            double rbar = 0.5 * (rj + rk);
            int base = 64 + 32 * pair_type(sp[j], sp[k]);
            for (int m = 0; m < NSHELL; ++m) {
                double x = rbar - shell_centre(m);
                double B = exp(-ETA_ANG * x * x);
                for (int nn = 0; nn < NSECTOR; ++nn) {
                    double A = pow(1.0 + cp * cos(sector_centre(nn)) + sp_ * sin(sector_centre(nn)), ZETA);
                    G[base + 8 * m + nn] += w * A * B;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ O5 --- */

static double celu(double z) { return (z > 0.0 ? z : 0.0) + fmin(0.0, CELU_ALPHA * (exp(z / CELU_ALPHA) - 1.0)); }
static double celu_deriv(double z) { return z > 0.0 ? 1.0 : exp(z / CELU_ALPHA); }

/* y[o] = sum_i W[o][i] x[i] + b[o] */
static void linear(const float* W, const float* b, int nout, int nin, const double* x, double* y)
{
    for (int o = 0; o < nout; ++o) {
        double s = 0.0;
        for (int i = 0; i < nin; ++i) s += (double)W[(size_t)o * nin + i] * x[i];
        y[o] = s + (double)b[o];
    }
}

/* g[i] = sum_o W[o][i] d[o] */
static void linear_t(const float* W, int nout, int nin, const double* d, double* g)
{
    for (int i = 0; i < nin; ++i) g[i] = 0.0;
    for (int o = 0; o < nout; ++o)
        for (int i = 0; i < nin; ++i) g[i] += (double)W[(size_t)o * nin + i] * d[o];
}

/* Energy of one atom of element e and, if dEdG != NULL, its gradient with
 * respect to the 384 input features. */
void oracle_mlp(int e, const float* weights, const double* G, double* E, double* dEdG)
{
    const float* p = weights + (size_t)e * PER_ELEMENT;
    const float *W1 = p, *b1 = W1 + H1 * NFEAT;
    const float *W2 = b1 + H1, *b2 = W2 + H2 * H1;
    const float *W3 = b2 + H2, *b3 = W3 + H3 * H2;
    const float *W4 = b3 + H3, *b4 = W4 + H3;
    double z1[H1], h1[H1], z2[H2], h2[H2], z3[H3], h3[H3], out;
    linear(W1, b1, H1, NFEAT, G, z1);
    for (int i = 0; i < H1; ++i) h1[i] = celu(z1[i]);
    linear(W2, b2, H2, H1, h1, z2);
    for (int i = 0; i < H2; ++i) h2[i] = celu(z2[i]);
    linear(W3, b3, H3, H2, h2, z3);
    for (int i = 0; i < H3; ++i) h3[i] = celu(z3[i]);
    linear(W4, b4, 1, H3, h3, &out);
    *E = out;
    if (!dEdG) return;
    double d3[H3], d2[H2], d1[H1], one = 1.0;
    linear_t(W4, 1, H3, &one, d3);
    for (int i = 0; i < H3; ++i) d3[i] *= celu_deriv(z3[i]);
    linear_t(W3, H3, H2, d3, d2);
    for (int i = 0; i < H2; ++i) d2[i] *= celu_deriv(z2[i]);
    linear_t(W2, H2, H1, d2, d1);
    for (int i = 0; i < H1; ++i) d1[i] *= celu_deriv(z1[i]);
    linear_t(W1, H1, NFEAT, d1, dEdG);
}

/* ------------------------------------------------------------------ O7 --- */

/* Adds dE_i/dx_a to out[3], given g = dE_i/dG_i. */
static void dEi_dxa(const double* pos, const int* sp, const nlist* L, int i, const double* g, int a,
                    double out[3])
{
    int self = (a == i);
    /* radial pairs */
    for (int t = L->start[i]; t < L->start[i + 1]; ++t) {
        int j = L->idx[t];
        if (!self && j != a) continue;
        double d[3];
        double r = dist(pos, i, j, d);
        double f = cutoff(r, RC_RAD), df = cutoff_deriv(r, RC_RAD);
        double dEdr = 0.0;
        for (int k = 0; k < NRAD; ++k) {
            double x = r - radial_centre(k);
            double ex = exp(-ETA_RAD * x * x);
            dEdr += g[NRAD * sp[j] + k] * ex * (df - 2.0 * ETA_RAD * x * f);
        }
        double s = (j == a ? 1.0 : 0.0) - (self ? 1.0 : 0.0);
        for (int c = 0; c < 3; ++c) out[c] += s * dEdr * d[c] / r;
    }
    /* angular triples */
    for (int ta = L->start[i]; ta < L->start[i + 1]; ++ta) {
        int j = L->idx[ta];
        double dj[3];
        double rj = dist(pos, i, j, dj);
        if (!(rj < RC_ANG)) continue;
        for (int tb = ta + 1; tb < L->start[i + 1]; ++tb) {
            int k = L->idx[tb];
            if (!self && j != a && k != a) continue;
            double dk[3];
            double rk = dist(pos, i, k, dk);
            if (!(rk < RC_ANG)) continue;
            double uj[3], uk[3];
            for (int c = 0; c < 3; ++c) { uj[c] = dj[c] / rj; uk[c] = dk[c] / rk; }
            double cs = uj[0] * uk[0] + uj[1] * uk[1] + uj[2] * uk[2];
            double cp = COS_SCALE * cs;
            double sq = sqrt(1.0 - cp * cp);
            double fj = cutoff(rj, RC_ANG), fk = cutoff(rk, RC_ANG);
            double dfj = cutoff_deriv(rj, RC_ANG), dfk = cutoff_deriv(rk, RC_ANG);
            double pre = ldexp(1.0, 1 - (int)ZETA);
            double rbar = 0.5 * (rj + rk);
            int base = 64 + 32 * pair_type(sp[j], sp[k]);
            double dE_dcp = 0.0, dE_drj = 0.0, dE_drk = 0.0;
            for (int m = 0; m < NSHELL; ++m) {
                double x = rbar - shell_centre(m);
                double B = exp(-ETA_ANG * x * x);
                double dB = -2.0 * ETA_ANG * x * B; /* dB/d rbar */
                for (int nn = 0; nn < NSECTOR; ++nn) {
                    double ct = cos(sector_centre(nn)), st = sin(sector_centre(nn));
                    double u = 1.0 + cp * ct + sq * st;
                    double A = pow(u, ZETA);
                    double dA = ZETA * pow(u, ZETA - 1.0) * (ct - cp * st / sq);
                    double gv = g[base + 8 * m + nn] * pre;
                    dE_dcp += gv * dA * B * fj * fk;
                    dE_drj += gv * A * (dB * 0.5 * fj * fk + B * dfj * fk);
                    dE_drk += gv * A * (dB * 0.5 * fj * fk + B * fj * dfk);
                }
            }
            double dE_dc = COS_SCALE * dE_dcp;
            double gj[3], gk[3];
            for (int c = 0; c < 3; ++c) {
                gj[c] = dE_drj * uj[c] + dE_dc * (uk[c] - cs * uj[c]) / rj;
                gk[c] = dE_drk * uk[c] + dE_dc * (uj[c] - cs * uk[c]) / rk;
            }
            for (int c = 0; c < 3; ++c) {
                if (j == a) out[c] += gj[c];
                if (k == a) out[c] += gk[c];
                if (self) out[c] -= gj[c] + gk[c];
            }
        }
    }
}

/* ------------------------------------------------------ public entries --- */

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Descriptors of every atom: G[n][384]. */
void oracle_descriptors(int n, const double* pos, const int* sp, double* G)
{
    nlist L;
    nlist_build(&L, n, pos);
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n; ++i) descriptor(pos, sp, &L, i, G + (size_t)i * NFEAT);
    nlist_free(&L);
}

/* Energy of one molecule.  Ei[n] (optional) receives per-atom energies and
 * F[n][3] (optional) the forces.  Returns E = sum_i E_i. */
double oracle_energy_forces(int n, const double* pos, const int* sp, const float* weights, double* Ei,
                            double* F)
{
    nlist L;
    nlist_build(&L, n, pos);
    double* e = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* g = F ? (double*)malloc(sizeof(double) * (size_t)n * NFEAT) : NULL;
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n; ++i) {
        double G[NFEAT];
        descriptor(pos, sp, &L, i, G);
        oracle_mlp(sp[i], weights, G, &e[i], g ? g + (size_t)i * NFEAT : NULL);
    }
    if (F) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int a = 0; a < n; ++a) {
            double acc[3] = {0.0, 0.0, 0.0};
            dEi_dxa(pos, sp, &L, a, g + (size_t)a * NFEAT, a, acc);
            for (int t = L.start[a]; t < L.start[a + 1]; ++t) {
                int i = L.idx[t];
                dEi_dxa(pos, sp, &L, i, g + (size_t)i * NFEAT, a, acc);
            }
            for (int c = 0; c < 3; ++c) F[3 * a + c] = -acc[c];
        }
    }
    double E = 0.0;
    for (int i = 0; i < n; ++i) E += e[i];
    if (Ei) memcpy(Ei, e, sizeof(double) * (size_t)n);
    free(e);
    free(g);
    nlist_free(&L);
    return E;
}

/* Forces on the selected atoms only: F_sel[nsel][3]. */
void oracle_forces_on(int n, const double* pos, const int* sp, const float* weights, int nsel, const int* sel,
                      double* F_sel)
{
    nlist L;
    nlist_build(&L, n, pos);
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < nsel; ++q) {
        int a = sel[q];
        double acc[3] = {0.0, 0.0, 0.0};
        double G[NFEAT], g[NFEAT], Ea;
        descriptor(pos, sp, &L, a, G);
        oracle_mlp(sp[a], weights, G, &Ea, g);
        dEi_dxa(pos, sp, &L, a, g, a, acc);
        for (int t = L.start[a]; t < L.start[a + 1]; ++t) {
            int i = L.idx[t];
            double Ei;
            descriptor(pos, sp, &L, i, G);
            oracle_mlp(sp[i], weights, G, &Ei, g);
            dEi_dxa(pos, sp, &L, i, g, a, acc);
        }
        for (int c = 0; c < 3; ++c) F_sel[3 * q + c] = -acc[c];
    }
    nlist_free(&L);
}

/* Harmonic test model of the paper's Methods example: E = sum of x^2. */
static double harmonic(int n, const double* x, double* F)
{
    double E = 0.0;
    for (int i = 0; i < 3 * n; ++i) {
        E += x[i] * x[i];
        F[i] = -2.0 * x[i];
    }
    return E;
}

static double kinetic(int n, const double* v, const double* m)
{
    double K = 0.0;
    for (int i = 0; i < n; ++i)
        K += 0.5 * m[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]) / KAPPA;
    return K;
}

/* Force model of the integrators: 0 network, 1 harmonic sum(x^2), 2 none,
 * 3 network plus harmonic (two force providers whose energies and forces add). */
static double model_forces(int model, int n, const double* x, const int* sp, const float* weights, double* F)
{
    if (model == 1) return harmonic(n, x, F);
    if (model == 2) {
        memset(F, 0, sizeof(double) * 3 * (size_t)n);
        return 0.0;
    }
    double E = oracle_energy_forces(n, x, sp, weights, NULL, F);
    if (model == 3) {
        double* Fh = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
        E += harmonic(n, x, Fh);
        for (int i = 0; i < 3 * n; ++i) F[i] += Fh[i];
        free(Fh);
    }
    return E;
}

/* O8: nsteps of NVE velocity Verlet on one molecule, in place on x and v
 * (both [n][3]).  model: see model_forces.
 * U[nsteps+1] and K[nsteps+1] (optional) receive the potential and kinetic
 * energy before the first step and after every step. */
void oracle_vv(int n, double* x, double* v, const double* m, const int* sp, const float* weights, int model,
               double dt, int nsteps, double* U, double* K)
{
    double* F = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double E = model_forces(model, n, x, sp, weights, F);
    if (U) U[0] = E;
    if (K) K[0] = kinetic(n, v, m);
    for (int s = 1; s <= nsteps; ++s) {
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) {
                v[3 * i + c] += 0.5 * dt * KAPPA * F[3 * i + c] / m[i];
                x[3 * i + c] += dt * v[3 * i + c];
            }
        E = model_forces(model, n, x, sp, weights, F);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) v[3 * i + c] += 0.5 * dt * KAPPA * F[3 * i + c] / m[i];
        if (U) U[s] = E;
        if (K) K[s] = kinetic(n, v, m);
    }
    free(F);
}

/* O10: Philox4x64-10.  Each of the ten rounds multiplies counter words 0 and
 * 2 by the two round constants (full 128-bit products), swaps the halves
 * across the two lanes and mixes in the key; the key advances by the two
 * Weyl constants between rounds. */
void oracle_philox4x64(const uint64_t* ctr, const uint64_t* key, uint64_t* out)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        const unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        const unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* O10: the three standard normal values of atom `atom` in step `step`. */
void oracle_langevin_noise(uint64_t seed, int64_t atom, int64_t step, double* z)
{
    const uint64_t ctr[4] = {(uint64_t)atom, (uint64_t)step, 0, 0};
    const uint64_t key[2] = {seed, 0};
    uint64_t w[4];
    oracle_philox4x64(ctr, key, w);
    double u[4];
    for (int q = 0; q < 4; ++q) u[q] = ((double)(w[q] >> 11) + 0.5) * ldexp(1.0, -53);
    const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    z[0] = r0 * cos(2.0 * PI * u[1]);
    z[1] = r0 * sin(2.0 * PI * u[1]);
    z[2] = r1 * cos(2.0 * PI * u[3]);
}

/* O9: nsteps of BAOAB Langevin dynamics on one molecule, in place on x and v.
 * Atom i draws its noise as caller index first_index + i; the first step
 * taken is step count first_step.  friction in 1/ps, temperature in K.
 * U and K as for oracle_vv. */
void oracle_langevin(int n, double* x, double* v, const double* m, const int* sp, const float* weights, int model,
                     double dt, int nsteps, double temperature, double friction, uint64_t seed, int64_t first_index,
                     int64_t first_step, double* U, double* K)
{
    double* F = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    const double a = exp(-friction * 1e-3 * dt);
    double E = model_forces(model, n, x, sp, weights, F);
    if (U) U[0] = E;
    if (K) K[0] = kinetic(n, v, m);
    for (int s = 1; s <= nsteps; ++s) {
        for (int i = 0; i < n; ++i) {
            double z[3];
            oracle_langevin_noise(seed, first_index + i, first_step + s - 1, z);
            const double sigma = sqrt((1.0 - a * a) * KB * temperature * KAPPA / m[i]);
            for (int c = 0; c < 3; ++c) {
                double* vi = &v[3 * i + c];
                double* xi = &x[3 * i + c];
                *vi += 0.5 * dt * KAPPA * F[3 * i + c] / m[i]; /* B */
                *xi += 0.5 * dt * *vi;                         /* A */
                *vi = a * *vi + sigma * z[c];                  /* O */
                *xi += 0.5 * dt * *vi;                         /* A */
            }
        }
        E = model_forces(model, n, x, sp, weights, F);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) v[3 * i + c] += 0.5 * dt * KAPPA * F[3 * i + c] / m[i]; /* B */
        if (U) U[s] = E;
        if (K) K[s] = kinetic(n, v, m);
    }
    free(F);
}
