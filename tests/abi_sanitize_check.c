/*
 * abi_sanitize_check.c -- a host-only driver of the library's C ABI for a
 * build whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers_cpu.py): parameter
 * validation on every rejected field, null-context calls, and the host E4M3
 * encoder over every float class.  It needs no GPU (nothing here reaches
 * device work; a valid nnp_create without a device fails cleanly).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nnp.h"

#define NW (4 * 94689)

static int fails = 0;
static void expect(int cond, const char* what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++fails;
    }
}

int main(void)
{
    enum { N = 6 };
    int32_t sp[N] = {0, 1, 2, 3, 0, 1};
    double m[N] = {1.008, 12.011, 14.007, 15.999, 1.008, 12.011};
    int32_t off[3] = {0, 4, N};
    float* w = calloc(NW, sizeof(float));
    nnp_params p;
    memset(&p, 0, sizeof p);
    p.n_atoms = N;
    p.n_molecules = 2;
    p.mol_offsets = off;
    p.species = sp;
    p.masses = m;
    p.weights = w;
    p.weights_count = NW;
    p.mlp_dtype = NNP_MLP_BF16_SPLIT;
    p.path = NNP_PATH_FUSED;
    p.return_mode = NNP_RETURN_ENERGY_FORCES;
    p.rebuild_every = 20;
    p.skin = 1.0;
    nnp_context* c = NULL;
    /* each invalid field alone */
    nnp_params q;
#define BAD(field, value)                                            \
    q = p;                                                           \
    q.field = value;                                                 \
    expect(nnp_create(&q, &c) == NNP_ERR_ARG && c == NULL, #field);
    BAD(n_atoms, 0)
    BAD(n_molecules, 0)
    BAD(n_molecules, N + 1)
    BAD(weights_count, 10)
    BAD(mlp_dtype, (nnp_dtype)9)
    BAD(path, (nnp_path)4)
    BAD(network_tile, 24)
    BAD(return_mode, (nnp_return)2)
    BAD(rebuild_every, 0)
    BAD(skin, -0.5)
    BAD(skin, NAN)
    BAD(max_neighbors, 257)
    BAD(atoms_per_tile, 11)
    BAD(species, NULL)
    BAD(masses, NULL)
    BAD(weights, NULL)
    BAD(mol_offsets, NULL)
    int32_t bad_off[3] = {0, 5, 4};
    BAD(mol_offsets, bad_off)
    int32_t bad_sp[N] = {0, 1, 2, 4, 0, 1};
    BAD(species, bad_sp)
    double bad_m[N] = {1.0, 1.0, -1.0, 1.0, 1.0, 1.0};
    BAD(masses, bad_m)
    expect(nnp_create(NULL, &c) == NNP_ERR_ARG, "null params");
    expect(nnp_create(&p, NULL) == NNP_ERR_ARG, "null out");
    w[17] = INFINITY;
    expect(nnp_create(&p, &c) == NNP_ERR_NONFINITE && c == NULL, "non-finite weight");
    w[17] = 0.0f;
    /* null context */
    double pos[3 * N] = {0}, e[2];
    expect(nnp_compute(NULL, pos, NULL, e, NULL) == NNP_ERR_ARG, "compute null");
    expect(nnp_step(NULL, 0.5, 1, 1) == NNP_ERR_ARG, "step null");
    expect(nnp_capture(NULL, 0.5, 1) == NNP_ERR_ARG, "capture null");
    expect(nnp_set_state(NULL, pos, NULL) == NNP_ERR_ARG, "set_state null");
    expect(nnp_get_state(NULL, pos, NULL, NULL, NULL, NULL) == NNP_ERR_ARG, "get_state null");
    expect(nnp_autotune(NULL, NULL, NULL) == NNP_ERR_ARG, "autotune null");
    int32_t cfg[3];
    expect(nnp_get_config(NULL, cfg) == NNP_ERR_ARG, "get_config null");
    expect(strcmp(nnp_last_error(NULL), "null context") == 0, "last_error null");
    for (int s = 0; s <= 7; ++s) expect(nnp_status_string((nnp_status)s) != NULL, "status string");
    nnp_destroy(NULL);
    /* the host E4M3 encoder over zeros, subnormals, normals, ties, saturation, NaN */
    enum { K = 4096 };
    float x[K];
    uint8_t host[K];
    for (int i = 0; i < K; ++i) x[i] = (float)ldexp((double)(i % 97) - 48.0, (i % 41) - 25);
    x[0] = 0.0f, x[1] = -0.0f, x[2] = NAN, x[3] = INFINITY, x[4] = -INFINITY, x[5] = 448.0f, x[6] = 464.0f;
    expect(nnp_debug_fp8_encode(x, K, NULL, host) == NNP_OK, "fp8 host encode");
    expect(host[5] == 0x7e && host[6] == 0x7e && host[2] == 0x7f, "fp8 saturation / NaN");
    expect(nnp_debug_fp8_encode(x, 0, NULL, host) == NNP_ERR_ARG, "fp8 n = 0");
    /* a valid context: created on a GPU, a clean HIP error without one */
    nnp_status s = nnp_create(&p, &c);
    expect(s == NNP_OK || s == NNP_ERR_HIP || s == NNP_ERR_OOM, "valid create");
    if (s == NNP_OK) nnp_destroy(c);
    free(w);
    printf("abi_sanitize_check %s (create: %s)\n", fails ? "FAILED" : "ok", nnp_status_string(s));
    return fails ? 1 : 0;
}
