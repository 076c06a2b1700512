/*
 * sanitize_check.c -- TEST INFRASTRUCTURE ONLY: a driver that calls every
 * entry point of nnp_oracle.c on small molecules and their edge cases, so
 * that a build of the oracle with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers_cpu.py) reaches all of
 * its code: pair search, descriptors, network, energies and forces, forces
 * on selected atoms, velocity Verlet, Philox noise and BAOAB Langevin
 * dynamics.  Exits 0 after printing a checksum; any sanitizer report aborts.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

long oracle_pairs(int n, const double* pos, double rc, int* out_i, int* out_j, long cap);
void oracle_mlp(int e, const float* weights, const double* G, double* E, double* dEdG);
void oracle_descriptors(int n, const double* pos, const int* sp, double* G);
double oracle_energy_forces(int n, const double* pos, const int* sp, const float* weights, double* Ei, double* F);
void oracle_forces_on(int n, const double* pos, const int* sp, const float* weights, int nsel, const int* sel,
                      double* F);
void oracle_vv(int n, double* x, double* v, const double* m, const int* sp, const float* weights, int model,
               double dt, int nsteps, double* U, double* K);
void oracle_philox4x64(const uint64_t* ctr, const uint64_t* key, uint64_t* out);
void oracle_langevin_noise(uint64_t seed, int64_t atom, int64_t step, double* z);
void oracle_langevin(int n, double* x, double* v, const double* m, const int* sp, const float* weights, int model,
                     double dt, int nsteps, double temperature, double friction, uint64_t seed, int64_t first_index,
                     int64_t first_step, double* U, double* K);
void oracle_set_threads(int t);

#define NW (4 * 94689)
#define NFEAT 384

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static double uni(void)  /* xorshift64*, uniform in [0, 1) */
{
    rs ^= rs >> 12;
    rs ^= rs << 25;
    rs ^= rs >> 27;
    return (double)((rs * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0);
}

static double sum;

static void run(int n, const double* pos, const int* sp, const float* w)
{
    double* G = malloc(sizeof(double) * NFEAT * (size_t)(n > 0 ? n : 1));
    double* Ei = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* F = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double* x = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double* v = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double* m = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int* sel = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    double U[6], K[6];
    long np = oracle_pairs(n, pos, 5.2, NULL, NULL, 0);
    int* pi = malloc(sizeof(int) * (size_t)(np > 0 ? np : 1));
    int* pj = malloc(sizeof(int) * (size_t)(np > 0 ? np : 1));
    oracle_pairs(n, pos, 5.2, pi, pj, np);
    oracle_descriptors(n, pos, sp, G);
    sum += oracle_energy_forces(n, pos, sp, w, Ei, F);
    sum += oracle_energy_forces(n, pos, sp, w, Ei, NULL);
    for (int i = 0; i < n; ++i) sel[i] = n - 1 - i;
    oracle_forces_on(n, pos, sp, w, n, sel, F);
    for (int i = 0; i < 3 * n; ++i) {
        x[i] = pos[i];
        v[i] = 0.01 * (uni() - 0.5);
    }
    for (int i = 0; i < n; ++i) m[i] = 1.0 + 14.0 * (double)sp[i];
    for (int model = 0; model < 4; ++model) oracle_vv(n, x, v, m, sp, w, model, 0.5, 5, U, K);
    oracle_langevin(n, x, v, m, sp, w, 0, 0.5, 5, 300.0, 0.1, 7u, 3, 11, U, K);
    oracle_langevin(n, x, v, m, sp, w, 1, 0.5, 5, 300.0, 50.0, 7u, 0, 0, NULL, NULL);
    for (int i = 0; i < n; ++i) sum += Ei[i] + F[3 * i] + x[3 * i];
    for (long q = 0; q < np; ++q) sum += 1e-9 * (pi[q] + pj[q]);
    free(G), free(Ei), free(F), free(x), free(v), free(m), free(sel), free(pi), free(pj);
}

int main(void)
{
    float* w = malloc(sizeof(float) * NW);
    for (int i = 0; i < NW; ++i) w[i] = (float)(0.2 * (uni() - 0.5));
    oracle_set_threads(2);
    /* 40 atoms of all four elements, random in a 7 A cube, kept >= 0.9 A apart */
    enum { N = 40 };
    double pos[3 * N];
    int sp[N];
    for (int i = 0; i < N;) {
        for (int c = 0; c < 3; ++c) pos[3 * i + c] = 7.0 * uni();
        int ok = 1;
        for (int j = 0; j < i && ok; ++j) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) d2 += (pos[3 * i + c] - pos[3 * j + c]) * (pos[3 * i + c] - pos[3 * j + c]);
            ok = d2 >= 0.81;
        }
        if (ok) {
            sp[i] = i % 4;
            ++i;
        }
    }
    run(N, pos, sp, w);
    /* edge cases: one atom, a dimer at the radial cutoff, a collinear and a
     * right-angle trimer inside the angular cutoff, no atoms at all */
    const double one[3] = {1.0, 2.0, 3.0};
    const int s1[1] = {3};
    run(1, one, s1, w);
    const double dim[6] = {0.0, 0.0, 0.0, 5.2, 0.0, 0.0};
    const int s2[2] = {0, 1};
    run(2, dim, s2, w);
    const double lin[9] = {0.0, 0.0, 0.0, 1.1, 0.0, 0.0, -1.3, 0.0, 0.0};
    const double rt[9] = {0.0, 0.0, 0.0, 1.1, 0.0, 0.0, 0.0, 1.3, 0.0};
    const int s3[3] = {2, 0, 3};
    run(3, lin, s3, w);
    run(3, rt, s3, w);
    run(0, NULL, NULL, w);
    double G[NFEAT], E, g[NFEAT];
    for (int f = 0; f < NFEAT; ++f) G[f] = uni();
    for (int e = 0; e < 4; ++e) {
        oracle_mlp(e, w, G, &E, g);
        sum += E + g[0];
    }
    uint64_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    oracle_philox4x64(ctr, key, out);
    double z[3];
    oracle_langevin_noise(9u, 100, 200, z);
    sum += (double)(out[0] >> 40) + z[0];
    free(w);
    printf("sanitize_check ok %.6e\n", sum);
    return isfinite(sum) ? 0 : 1;
}
