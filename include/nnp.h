/*
 * nnp.h -- C ABI of the MI355X (gfx950) gas-phase NNP energy/force/MD library.
 *
 * The library implements the force-provider contract of the paper (Methods
 * section: a model object registered with the MD engine, called with the
 * positions, returning the potential energy, with the forces obtained as
 * minus its gradient; the explicit-force provider variant returns both):
 *
 *     nnp_create(params)  ->  nnp_compute(positions, box)  ->  energy, forces
 *                         ->  nnp_step(dt, n)              (NVE velocity Verlet, or
 *                                                           Langevin: nnp_set_thermostat)
 *
 * The model is a symmetry-function network potential:
 *   - pair sets within 5.2 A (radial) and 3.5 A (angular), gas phase or an
 *     orthorhombic periodic box (nearest images; nnp_set_box);
 *   - 64 radial features (16 Gaussians, eta = 16 A^-2, centres 0.9..5.1 A, cosine
 *     cutoff 5.2 A, per neighbour element) and 320 angular features (4 shells x 8
 *     sectors, zeta = 32, cosine cutoff 3.5 A, per unordered element pair);
 *   - per-element network 384 -> 160 -> 128 -> 96 -> 1 with CELU(alpha = 0.1);
 *   - E = sum_i E_i, forces F = -dE/dx by a hand-written adjoint;
 *   - FP64 energy reduction and FP64 velocity Verlet (the paper's engine keeps
 *     integration in higher precision than the model, Results section).
 *
 * Units: Angstrom, fs, amu, eV.  Elements: 0 = H, 1 = C, 2 = N, 3 = O.
 *
 * Ownership: the caller owns every array it passes.  Host arrays are copied
 * during the call; no caller pointer is retained after a call returns (the
 * paper's keep-alive rule for the registered model object is replaced by the
 * opaque context, which the caller keeps until nnp_destroy).  The context owns
 * all device memory, streams it created, and captured graphs.  Functions that
 * take device pointers borrow them for the duration of the work they enqueue
 * on the context stream.
 *
 * Errors: every call returns an nnp_status; no C++ exception crosses this
 * boundary.  Arguments are validated on the host before any device work; a
 * failed validation leaves the context unchanged.  nnp_last_error() gives a
 * per-context message for the most recent failure.
 *
 * Threading: a context may be used by one host thread at a time; distinct
 * contexts are independent.
 */
#ifndef NNP_H
#define NNP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnp_context nnp_context;

typedef enum {
    NNP_OK = 0,
    NNP_ERR_ARG = 1,         /* invalid argument (NULL, out of range, size mismatch) */
    NNP_ERR_NONFINITE = 2,   /* NaN/Inf input, coincident atoms, or non-finite result */
    NNP_ERR_UNSUPPORTED = 3, /* valid request the library does not implement (e.g. a box) */
    NNP_ERR_OOM = 4,         /* device allocation failed */
    NNP_ERR_HIP = 5,         /* HIP runtime error; message holds the HIP error string */
    NNP_ERR_STATE = 6        /* call not valid in the current state, or a device-side
                                capacity overflow (neighbour list, LDS environment) */
} nnp_status;

/* What nnp_compute and nnp_compute_device return (the paper's return flag of
 * a registered Python callable, Methods section: the energy alone, the engine
 * then obtaining the forces by differentiating it, or the energy together
 * with explicit forces).
 *   NNP_RETURN_ENERGY_FORCES  energy and forces (0 selects this);
 *   NNP_RETURN_ENERGY         energy only: the evaluation runs the network
 *                             forward alone (no input gradient, no adjoint),
 *                             leaves the context's forces untouched, and a
 *                             non-NULL forces argument is NNP_ERR_ARG.  Forces
 *                             then come from differentiation: nnp_forces_device
 *                             after nnp_energy_device, or the adjoint inside
 *                             nnp_step (MD always needs them). */
typedef enum { NNP_RETURN_ENERGY = 1, NNP_RETURN_ENERGY_FORCES = 3 } nnp_return;

/* Arithmetic of the network GEMMs.  Descriptors and the adjoint are FP32 in
 * every mode; energy reduction and integration are FP64.
 *   NNP_MLP_FP32        FP32 FMA on the vector ALUs;
 *   NNP_MLP_BF16        BF16 MFMA, FP32 accumulation, one product per GEMM;
 *   NNP_MLP_FP8         OCP FP8 E4M3 MFMA, FP32 accumulation: weights scaled per
 *                       matrix by 448 / amax|W| (static), every other operand per
 *                       tile and layer by 448 / amax of the tile (no saturation);
 *   NNP_MLP_BF16_SPLIT  BF16 MFMA on split operands: each FP32 weight and
 *                       activation x = hi + lo with hi = bf16(x), lo = bf16(x - hi);
 *                       hi*hi + hi*lo + lo*hi, FP32 accumulation (three MFMAs). */
typedef enum { NNP_MLP_FP32 = 0, NNP_MLP_BF16 = 1, NNP_MLP_FP8 = 2, NNP_MLP_BF16_SPLIT = 3 } nnp_dtype;

/* Kernel organisation of one energy/force evaluation.
 *   NNP_PATH_PLAIN: one kernel per stage (pair list, descriptors, network,
 *                   adjoint), descriptors and dE/dG round-trip through HBM;
 *   NNP_PATH_FUSED: one kernel per evaluation; a workgroup takes a tile of
 *                   atoms of one element through descriptors, network and
 *                   adjoint with every intermediate held in LDS;
 *   NNP_PATH_SPLIT: three kernels: descriptors of small tiles (pooled angular
 *                   work) -> G in HBM; the network over wide tiles of up to
 *                   network_tile atoms of one element, each weight fragment
 *                   serving all of them -> dE/dG in HBM; the adjoint of the
 *                   small tiles.  BF16 and split-BF16 networks only (else
 *                   NNP_ERR_UNSUPPORTED at creation).  Built for large
 *                   systems, where the fused kernel's per-tile weight reads
 *                   and its one workgroup per compute unit bound throughput. */
typedef enum { NNP_PATH_PLAIN = 0, NNP_PATH_FUSED = 1, NNP_PATH_SPLIT = 2 } nnp_path;

typedef struct {
    int32_t n_atoms;             /* total atoms over all molecules, > 0 */
    int32_t n_molecules;         /* >= 1; molecules never interact */
    const int32_t* mol_offsets;  /* [n_molecules + 1], molecule m = atoms
                                    [off[m], off[m+1]); NULL allowed iff n_molecules == 1 */
    const int32_t* species;      /* [n_atoms], each in {0, 1, 2, 3} */
    const double* masses;        /* [n_atoms] amu, each > 0 */
    const float* weights;        /* network blob, float32, per element H, C, N, O:
                                    W1[160][384] b1[160] W2[128][160] b2[128]
                                    W3[96][128] b3[96] W4[1][96] b4[1] */
    size_t weights_count;        /* number of floats in the blob (4 * 94689) */
    nnp_dtype mlp_dtype;
    nnp_path path;
    nnp_return return_mode;      /* 0 or NNP_RETURN_ENERGY_FORCES, or NNP_RETURN_ENERGY */
    int32_t rebuild_every;       /* pair-list rebuild cadence in steps (e.g. 20), >= 1 */
    double skin;                 /* pair-list skin in A (e.g. 1.0), >= 0 */
    int32_t max_neighbors;       /* capacity of one atom's pair list (cutoff 5.2 + skin),
                                    <= 256; 0 selects 192 */
    int32_t atoms_per_tile;      /* atoms per workgroup: 4, 5, 8, 10, 12 to 15 or, with
                                    the BF16 and split-BF16 networks, 16 (fused path); 8 or
                                    16 (plain path); 4, 5, 7 or 10 (descriptor and adjoint
                                    kernels of the split path); 0 selects 16 (plain), 5
                                    (split) or, for the fused path, the smallest of 8, 10
                                    and 12 to 15 (16 with the BF16 networks) that gives at
                                    most one workgroup per compute unit, else the one of 10
                                    and 12 to 15 (16) with the least modelled time in
                                    rounds of one workgroup per compute unit */
    void* stream;                /* hipStream_t to run on (see use_stream) */
    int32_t use_stream;          /* nonzero: run on `stream` even when it is NULL (the null
                                    stream, e.g. PyTorch's default stream); zero: a NULL
                                    stream means a stream created and owned by the context.
                                    Multi-step graphs cannot be captured on the null stream:
                                    nnp_step then launches its kernels directly. */
    int32_t network_tile;        /* split path: atoms per workgroup of the network kernel,
                                    16, 32, 48 or 64; 0 selects 64.  Ignored by the other
                                    paths. */
} nnp_params;

/* Creates a context: validates params, sorts atoms into the internal order,
 * uploads weights and allocates every device buffer.  Positions and velocities
 * start at zero; call nnp_set_state or nnp_compute before nnp_step. */
nnp_status nnp_create(const nnp_params* params, nnp_context** out);

/* Releases the context and every device resource it owns.  NULL is a no-op. */
void nnp_destroy(nnp_context* ctx);

/* Energy (and forces) at the given positions (the force-provider call).
 *   pos     host [n_atoms][3] double, caller order.  Must be finite, no two
 *           atoms of one molecule closer than 1e-6 A (else NNP_ERR_NONFINITE);
 *   box     NULL keeps the context's box (gas phase unless nnp_set_box gave
 *           one); else host [3] double, the edges of an orthorhombic periodic
 *           box, which becomes the context's box as with nnp_set_box;
 *   energy  host [n_molecules] double, molecule potential energies (eV);
 *   forces  host [n_atoms][3] double (eV/A), or NULL.  With return_mode
 *           NNP_RETURN_ENERGY_FORCES the forces are computed either way (they
 *           become the context's forces for a following nnp_step); with
 *           NNP_RETURN_ENERGY only the energy is computed and forces must be
 *           NULL (else NNP_ERR_ARG).
 * The positions become the context's current positions (velocities are kept);
 * the pair list is rebuilt.  Synchronises the context stream. */
nnp_status nnp_compute(nnp_context* ctx, const double* pos, const double* box, double* energy,
                       double* forces);

/* Device-pointer form used by the PyTorch binding (autograd).  All pointers are
 * device memory, caller order, enqueued on the context stream, no host sync:
 *   d_pos     [n_atoms][3]; d_pos_is_f64 selects double (1) or float (0);
 *   d_energy  [n_molecules] double (written);
 *   d_forces  [n_atoms][3] double, or NULL for energy only (then the network
 *             backward and the adjoint are skipped); must be NULL with
 *             return_mode NNP_RETURN_ENERGY (else NNP_ERR_ARG).
 * No host-side validation of the device positions is possible; a non-finite
 * result is reported by the next host-synchronising call. */
nnp_status nnp_compute_device(nnp_context* ctx, const void* d_pos, int d_pos_is_f64, double* d_energy,
                              double* d_forces);

/* Differentiation entry points (the energy-only force-provider contract of the
 * paper's Methods section, where forces come from differentiating the energy).
 * Device pointers, caller order, context stream, no host sync.
 *
 * nnp_energy_device: energies [n_molecules] (double) at d_pos ([n_atoms][3],
 *   double if d_pos_is_f64 else float).  keep == 0 (recompute mode): only the
 *   pair list and the positions stay on the device.  keep != 0 (stored mode):
 *   the descriptors G and dE/dG ([n_atoms][384] float each) are also kept, at
 *   2 * 1536 bytes per atom of extra device memory (allocated on first use).
 * nnp_forces_device: forces [n_atoms][3] (double) at the positions of the
 *   last nnp_energy_device call: from the kept dE/dG through the adjoint
 *   alone (stored mode), or by recomputing descriptors, network forward and
 *   backward and the adjoint (recompute mode).  NNP_ERR_STATE without a
 *   preceding nnp_energy_device call. */
nnp_status nnp_energy_device(nnp_context* ctx, const void* d_pos, int d_pos_is_f64, double* d_energy, int keep);
nnp_status nnp_forces_device(nnp_context* ctx, double* d_forces);

/* Allocation-free stored mode, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): nnp_energy_device(ctx, d_pos, d_pos_is_f64, d_energy, 1) with
 * G and dE/dG kept in a static device array of the library instead of
 * context buffers allocated on first use.  The array holds at most 8,192
 * atoms ([2][8192][384] float, 24 MiB per GPU, held until the process ends);
 * a larger context gets NNP_ERR_ARG before any device work.  The call itself
 * allocates nothing (no hipMalloc, hipFree or allocating library routine);
 * its first call on a device looks up the array's address there.
 * nnp_forces_device then runs the adjoint from the array.  Every call on one
 * GPU, from any context, shares that GPU's array: a later call replaces the
 * kept G and dE/dG, after which nnp_forces_device of the earlier context
 * returns NNP_ERR_STATE; calls of different host threads or streams that
 * overlap on one GPU race.  Arguments, results and stream as for
 * nnp_energy_device. */
nnp_status nnp_energy_device_static(nnp_context* ctx, const void* d_pos, int d_pos_is_f64, double* d_energy);

/* Periodic boundary conditions (the force provider's compute(positions, box)
 * contract, Methods): box = host [3] double, the edges (A) of an orthorhombic
 * box with one corner at the origin, or NULL for the gas phase (the default).
 * Every displacement takes the nearest periodic image; positions are never
 * wrapped (MD keeps unwrapped coordinates).  Each edge must be finite and at
 * least 2 (5.2 + skin) A, so that every atom pair within the pair-list radius
 * has exactly one image in range (else NNP_ERR_ARG); the context must hold
 * one molecule (else NNP_ERR_UNSUPPORTED).  A molecule of more than 4,096
 * atoms uses a cell list tiling the box when every edge holds at least three
 * cells of 5.2 + skin A.  A new box invalidates the pair list and the
 * captured graphs; the next evaluation rebuilds.  Synchronises. */
nnp_status nnp_set_box(nnp_context* ctx, const double* box);

/* Sets positions and velocities (host [n_atoms][3] double, caller order;
 * either may be NULL to keep the current value). Forces are recomputed lazily. */
nnp_status nnp_set_state(nnp_context* ctx, const double* pos, const double* vel);

/* Copies the current state to the host.  Any pointer may be NULL.
 *   pos, vel, forces  [n_atoms][3] double, caller order;
 *   pot, kin          [n_molecules] double: potential and kinetic energy of the
 *                     most recent evaluated step.  Synchronises. */
nnp_status nnp_get_state(nnp_context* ctx, double* pos, double* vel, double* forces, double* pot,
                         double* kin);

/* Advances n_steps of NVE velocity Verlet with time step dt_fs:
 *   v += dt/2 kappa F/m;  x += dt v;  F = F(x);  v += dt/2 kappa F/m,
 * kappa = 9.64853321e-3 A fs^-2 per eV A^-1 amu^-1.  The pair list is rebuilt
 * every rebuild_every steps, and earlier when an atom moved more than skin/2
 * since the last rebuild (decided on the device; counted in nnp_stats).
 * use_graph != 0 replays the steps from a captured HIP graph (captured on
 * first use for the given block length and dt).  Returns after enqueueing;
 * nnp_get_state / nnp_energy_log synchronise. */
nnp_status nnp_step(nnp_context* ctx, double dt_fs, int32_t n_steps, int32_t use_graph);

/* Captures and instantiates the HIP graphs that nnp_step(ctx, dt_fs, n_steps,
 * 1) replays (one per block length: min(n_steps, 200) and the remainder),
 * without running any step, so that a following nnp_step with the same
 * arguments replays cached graphs only (serving loops, timed regions).
 * The state is unchanged.  NNP_ERR_STATE on the null stream or with extra
 * force providers registered (their steps are not captured). */
nnp_status nnp_capture(nnp_context* ctx, double dt_fs, int32_t n_steps);

/* Extra force providers (the paper's callback mechanism, Methods: the engine
 * calls back into caller code for energies and forces; its explicit-force
 * provider, AIMD section): after every network evaluation of nnp_compute,
 * nnp_compute_device (with forces) and nnp_step, each registered provider is
 * called on the host thread of that call as
 *   rc = fn(user, n_atoms, n_molecules, d_pos, d_forces, d_energy, stream)
 * with d_pos holding the current positions (caller order, [n_atoms][3]
 * double, A) and d_forces ([n_atoms][3] double) and d_energy ([n_molecules]
 * double) cleared; it enqueues work on `stream` (the context stream, a
 * hipStream_t) or works synchronously, leaving its forces (eV/A) and
 * per-molecule energies (eV) in those buffers, and returns 0 (anything else:
 * the calling function returns NNP_ERR_STATE; the evaluation is discarded,
 * and inside nnp_step the interrupted step leaves positions and velocities
 * mid-step: set the state again before stepping on).  The library adds them to the
 * network's forces (64-bit fixed point, 2^-32 eV/A, |component| < 2^15) and
 * molecule energies (not to the per-atom energies).  The three buffers are
 * caller-owned device memory and, like `user`, must stay valid until
 * nnp_clear_forces or nnp_destroy (the paper's keep-alive rule for the
 * registered model).  With providers registered nnp_step launches its kernels
 * step by step without graphs, and nnp_time_steps returns NNP_ERR_UNSUPPORTED.
 * At most 8 providers; NULL fn or buffers: NNP_ERR_ARG. */
typedef int (*nnp_force_fn)(void* user, int32_t n_atoms, int32_t n_molecules, const double* d_pos,
                            double* d_forces, double* d_energy, void* stream);
nnp_status nnp_add_force(nnp_context* ctx, nnp_force_fn fn, void* user, double* d_pos, double* d_forces,
                         double* d_energy);
/* Removes every extra force provider (synchronises the context stream). */
nnp_status nnp_clear_forces(nnp_context* ctx);

/* Thermostat of nnp_step (the paper times its runs with Langevin dynamics at
 * a friction of 0.1 ps^-1, Results section).  friction_per_ps > 0 makes every
 * following step a BAOAB Langevin step (Leimkuhler and Matthews 2013):
 *   v += dt/2 kappa F/m;  x += dt/2 v;
 *   v = a v + sqrt((1 - a^2) kB T kappa / m) z,  a = exp(-friction dt);
 *   x += dt/2 v;  F = F(x);  v += dt/2 kappa F/m,
 * with velocities (and the logged kinetic energy) at whole steps.  z holds
 * three standard normal values per atom and step: Philox4x64-10 (Salmon et al.,
 * SC'11) of the counter (caller atom index, step count, 0, 0) under the key
 * (seed, 0), each 64-bit word w taken as u = (floor(w / 2^11) + 1/2) 2^-53, and
 * Box-Muller on (u0, u1) and (u2, u3) giving sqrt(-2 ln u0) cos(2 pi u1),
 * sqrt(-2 ln u0) sin(2 pi u1), sqrt(-2 ln u2) cos(2 pi u3).  The step count is
 * the number of steps the context has taken (nnp_stats), so a trajectory is
 * reproducible from (state, step count, seed) and independent of graphs.
 *   temperature_K    >= 0 (kB = 8.617333262e-5 eV/K);
 *   friction_per_ps  >= 0; 0 (the default) restores NVE velocity Verlet;
 *   seed             any value.
 * Non-finite or negative values: NNP_ERR_ARG, settings unchanged. */
nnp_status nnp_set_thermostat(nnp_context* ctx, double temperature_K, double friction_per_ps, uint64_t seed);

/* Potential and kinetic energy of the last min(count, steps done, ring size)
 * steps, oldest first: U and K are [count][n_molecules] double.  Returns the
 * number of steps written in *written.  The ring holds 4096 steps.  Like
 * nnp_get_state, returns NNP_ERR_STATE (a capacity was exceeded) or
 * NNP_ERR_NONFINITE when a step since the flags were last clear produced
 * such a result, writing nothing (*written = 0). */
nnp_status nnp_energy_log(nnp_context* ctx, int32_t count, double* U, double* K, int32_t* written);

/* Counters since creation: [0] evaluations, [1] pair-list rebuilds, [2] rebuilds
 * forced by displacement > skin/2, [3] steps, [4] longest pair list, [5] most
 * neighbours within 5.2 A, [6] most neighbours within 3.5 A (capacities: 256,
 * 160 and 96 per atom; exceeding one makes nnp_compute, nnp_get_state,
 * nnp_energy_log and the timing calls return NNP_ERR_STATE from then on,
 * while nnp_stats keeps reporting these counters).  stats is int64[7]. */
nnp_status nnp_stats(nnp_context* ctx, int64_t* stats);

/* The kernel configuration in use: config[0] path (nnp_path), [1] atoms per
 * tile, [2] atoms per network tile of the split path.  With atoms_per_tile
 * 0 the fused path's tile size is chosen when the positions are first set
 * (see nnp_params.atoms_per_tile); nnp_autotune may change all three.
 * config is int32[3].  No device work. */
nnp_status nnp_get_config(const nnp_context* ctx, int32_t* config);

/* Descriptors at the given host positions, for parity checks: G is host
 * [n_atoms][384] float, caller order.  Synchronises. */
nnp_status nnp_debug_descriptors(nnp_context* ctx, const double* pos, float* G);

/* Per-atom energies E_i (host [n_atoms] double, caller order) of the most
 * recent evaluation.  Synchronises. */
nnp_status nnp_debug_atom_energies(nnp_context* ctx, double* Ei);

/* Bytes of device memory the context holds (buffers, weights, graphs' inputs). */
nnp_status nnp_device_bytes(nnp_context* ctx, int64_t* bytes);

/* Times the candidate kernel configurations on the current positions and
 * keeps the fastest:
 *   plain path: atoms per network tile 8 or 16;
 *   fused path, FP32 / FP8 networks: atoms per workgroup 4, 5, 8, 10 and
 *     12 to 15;
 *   fused or split path, BF16 / split-BF16 networks: the fused kernel with
 *     4, 5, 8, 10, 12 to 16 atoms per workgroup, and the split path
 *     with 4, 5, 7 or 10 atoms per descriptor / adjoint workgroup times 32 or
 *     64 atoms per network workgroup (the path may change between fused and
 *     split: same arithmetic, results equal to rounding).
 * If cache_path is not NULL the choice is read from / appended to that
 * JSON-lines file, keyed by the power-of-two buckets of the atom and molecule
 * counts, the path family, the network dtype and periodicity; a cached
 * choice is applied without timing.  choice (may be NULL) receives
 * {path, atoms_per_tile, network_tile, from_cache}.  Synchronises. */
nnp_status nnp_autotune(nnp_context* ctx, const char* cache_path, int32_t* choice);

/* Kernel timing on the context stream with HIP events, at the current
 * positions: runs one evaluation to make the pair list current, then times
 * reps back-to-back launches of the evaluation kernel(s) alone (the pair
 * list is not rebuilt during them) and reps launches of the force-gather /
 * energy kernel alone.  ms[0] and ms[1] receive the average milliseconds per
 * launch of each.  Used by the benchmark's roofline report.  Synchronises. */
nnp_status nnp_time_kernels(nnp_context* ctx, int32_t reps, double* ms);

/* Event-timed MD: runs n_steps velocity-Verlet steps like nnp_step without
 * a graph; every kernel dispatch of the evaluation and of the force-sum /
 * integration kernel carries HIP events that the dispatch itself stamps at
 * the start and the end of its execution (on the context stream).  ms[0]
 * receives the average milliseconds per step of the evaluation kernel(s)
 * (first dispatch start to last dispatch end), ms[1] that of the force-sum /
 * integration kernel, ms[2] the average time per step from the first
 * evaluation's start to the last integration's end.  The trajectory
 * advances exactly as with nnp_step (pair-list rebuilds included).  Used by
 * the benchmark's roofline report.  Synchronises; n_steps >= 1, dt > 0. */
nnp_status nnp_time_steps(nnp_context* ctx, double dt_fs, int32_t n_steps, double* ms);

/* E4M3 encodings of x[n]: host_out by the library's host encoder (used for
 * the weights), device_out by the device conversion instruction (used for
 * activations); either may be NULL.  A format check, no context needed. */
nnp_status nnp_debug_fp8_encode(const float* x, int32_t n, uint8_t* device_out, uint8_t* host_out);

/* Message for the most recent failure on this context ("" if none). */
const char* nnp_last_error(const nnp_context* ctx);

/* Static name of a status code. */
const char* nnp_status_string(nnp_status s);

#ifdef __cplusplus
}
#endif

#endif /* NNP_H */
