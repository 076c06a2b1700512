// nnp_internal.h -- device-side data layout shared by the HIP kernels and the
// host runtime of the NNP library (never exposed through the C ABI).
//
// Data layout in HBM (internal atom order: element-major H, C, N, O; within an
// element by molecule; within a molecule by a Morton key of the initial
// positions, so consecutive atoms of a tile are spatial neighbours):
//   pos    double4[n]    x, y, z (A), w = element as a double  (FP64 master)
//   vel    double4[n]    A/fs
//   frc    double4[n]    gathered FP64 forces (eV/A)
//   ref    float4[n]     positions at the last pair-list rebuild
//   nbr    int[n][cap]   pair list (cutoff 5.2 + skin), ascending internal index
//   facc   int64[kFaccCopies][n][4] force accumulators of the running evaluation, fixed
//                        point with 2^-32 eV/A resolution (x, y, z, unused),
//                        one copy per die (accelerator complex); integer
//                        addition makes the sum independent of the order of
//                        the atomic adds and of the copies
//   Ei     float[n]      per-atom energies of the last evaluation
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nnp {

constexpr int kNumSpecies = 4;
constexpr int kNumRadial = 16;
constexpr int kNumShells = 4;
constexpr int kNumSectors = 8;
constexpr int kNumFeat = 384;   // 4 * 16 radial + 10 * 32 angular
constexpr int kH1 = 160, kH2 = 128, kH3 = 96;

constexpr double kFixScale = 4294967296.0;  // fixed-point force units per eV/A (2^32)
// Largest accepted |force component| of one fixed-point term (2^15 eV/A).
// An atom's sum collects at most ~3.1e4 terms: up to 160 neighbours' energies
// with a radial term and an angular term of at most 95 adds each, its own
// energy's negated sum of the same, and up to 8 provider forces; 3.1e4 x 2^15
// x 2^32 < 2^62, so no sum (nor the copies' total) can wrap int64.  A larger
// term raises the non-finite flag instead of being added.
constexpr float kFixMax = 32768.0f;
constexpr float kCutRad = 5.2f;
constexpr float kCutAng = 3.5f;
constexpr float kEtaRad = 16.0f;
constexpr float kEtaAng = 8.0f;
constexpr float kCosScale = 0.95f;
constexpr float kCeluAlpha = 0.1f;
constexpr double kKappa = 9.64853321e-3;  // A fs^-2 per eV A^-1 amu^-1

constexpr int kRadMax = 160;  // radial entries per atom held in LDS
constexpr int kAngMax = 96;   // angular entries per atom held in LDS
constexpr int kCapMax = 256;  // largest pair-list capacity (slot fits in 8 bits)
constexpr int kRing = 4096;   // energy log ring (steps)
constexpr int kXcds = 8;      // accelerator complex dies; workgroups go round-robin
constexpr int kTileCap = 16;  // largest atoms-per-tile (MFMA columns)
constexpr int kSharedScanCap = 4096;  // molecule size up to which a tile's pair lists are rebuilt together
constexpr int kFaccCopies = 4;  // copies of the force sums: workgroup b adds into copy (b / 8) mod 4

// Per-element FP32 weight block (floats).  Forward dense layers read the
// transposed matrices ([in][out], coalesced over outputs), the backward ones
// the original [out][in] rows (coalesced over inputs).
struct W32Layout {
    static constexpr int Wt1 = 0;                    // [384][160]
    static constexpr int W1 = Wt1 + kNumFeat * kH1;  // [160][384]
    static constexpr int Wt2 = W1 + kH1 * kNumFeat;  // [160][128]
    static constexpr int W2 = Wt2 + kH1 * kH2;       // [128][160]
    static constexpr int Wt3 = W2 + kH2 * kH1;       // [128][96]
    static constexpr int W3 = Wt3 + kH2 * kH3;       // [96][128]
    static constexpr int W4 = W3 + kH3 * kH2;        // [96]
    static constexpr int B1 = W4 + kH3;              // [160]
    static constexpr int B2 = B1 + kH1;              // [128]
    static constexpr int B3 = B2 + kH2;              // [96]
    static constexpr int B4 = B3 + kH3;              // [1]
    static constexpr int Stride = ((B4 + 1 + 63) / 64) * 64;
};

// Per-element BF16 MFMA A-operand fragments (16 rows x 32 k per fragment,
// 64 lanes x 8 values).  Fragment (mt, kt) of a layer sits at
// base + mt * KT + kt.
struct FragLayout {
    static constexpr int F1 = 0;               // W1    M=160 K=384: 10 x 12
    static constexpr int F2 = F1 + 10 * 12;    // W2    M=128 K=160:  8 x 5
    static constexpr int F3 = F2 + 8 * 5;      // W3    M=96  K=128:  6 x 4
    static constexpr int B3 = F3 + 6 * 4;      // W3^T  M=128 K=96:   8 x 3
    static constexpr int B2 = B3 + 8 * 3;      // W2^T  M=160 K=128: 10 x 4
    static constexpr int B1 = B2 + 10 * 4;     // W1^T  M=384 K=160: 24 x 5
    static constexpr int Count = B1 + 24 * 5;  // 368 fragments per element
};

// Device step state.  Read by every workgroup of the integration kernel at
// its start and written by the workgroup whose arrival count shows that all
// of them have read it (it writes at its own end, nobody waits); read by
// every kernel of the next step.
constexpr int kArriveGroups = 8;      // arrival counters of the integration kernel's two-level count
constexpr int kArriveGroupMin = 128;  // workgroups from which it counts in two levels

struct StepState {
    int step;          // steps completed
    int age;           // evaluations since the last rebuild
    int lists_valid;   // 0 until the first build, and after positions are set from outside
    int viol[2];       // viol[n & 1]: an atom moved more than skin/2 before evaluation n
    int overflow;      // a capacity (pair list, radial or angular LDS entries) was exceeded
    int nonfinite;     // a non-finite energy or force was produced
    int last_slot;     // step index of the most recent evaluation (ring slot = index % kRing)
    unsigned started;  // workgroups (groups of them in large grids) of the running integration kernel
                       // that have read the state
    int max_ns, max_nr, max_na;  // largest pair-list / radial / angular count seen
    int pad;
    long long n_eval, n_rebuild, n_forced;
    // arrivals at the running integration kernel per group of workgroups
    // (workgroup b in group b mod kArriveGroups), counters 128 B apart
    alignas(128) unsigned arrive[kArriveGroups][32];
};

// Cell grid of one large molecule (cells of edge >= 5.2 + skin; atoms outside
// the grid are clamped into its boundary cells, which keeps every pair within
// the list cutoff in adjacent cells), or of the periodic box (cells tile the
// box; an atom's cell is that of its position wrapped into the box).
struct CellGrid {
    double ox, oy, oz;     // origin
    double ihx, ihy, ihz;  // 1 / cell edge per dimension
    int nx, ny, nz;        // cells per dimension (>= 3 each when periodic)
    int first;             // index of the grid's first cell in the global cell arrays
    int periodic;          // cells cover the periodic box and wrap around
};

struct Sys {
    int n, nmol, cap, ntiles;
    int ncells;        // cells over all grids (0: no cell lists)
    int rebuild_every;
    float rlist2;      // (5.2 + skin)^2
    float half_skin2;  // (skin / 2)^2
    double4* pos;
    double4* vel;
    double4* frc;
    float4* ref;
    // orthorhombic periodic box (one molecule); displacements take the nearest
    // image, positions are never wrapped
    int periodic;
    double3 box, ibox;  // edges (A) and their inverses
    // Langevin dynamics (BAOAB) of nnp_step; gamma == 0 selects velocity Verlet
    double gamma;        // friction (1/fs)
    double kT;           // thermostat temperature (eV)
    unsigned long long seed;  // Philox key of the thermostat noise
    const double* kinv;  // kappa / m
    const double* mass;
    const int* mol;
    const int2* mrange;  // [nmol * 4] internal index range of each element of a molecule
    const int4* tiles;      // {first atom of the initial tiling, count, element, 0}
    const int* tile_atoms;  // [ntiles][kTileCap] atom in each column of a tile
    const int* tile_mol;    // [ntiles] the molecule of all of a tile's atoms when it is scanned without a
                            // cell grid and has at most kSharedScanCap atoms, else -1
    // split evaluation: network tiles of up to 16 wide_blk consecutive atoms of
    // one element {first atom, count, element, 0}
    const int4* wtiles;
    int nwtiles, wide_blk;
    int* work;              // [n] angular pairs + radial entries / 2 at the last evaluation
    int* nbr;
    int* ncnt;
    unsigned long long* facc;  // [kFaccCopies][n][4] fixed-point forces, zero between evaluations
    float* Ei;
    double* Uring;  // [kRing][nmol]
    double* Kring;
    double* Eacc;   // [2][nmol] sums of evaluation n in Eacc[n & 1] (n = n_eval when it is gathered)
    double* Kacc;
    double* Ecur;   // [nmol] potential / kinetic energy of the most recent evaluation, after a flush
    double* Kcur;
    const int* perm;  // [n] internal -> caller index
    double* stage;    // [3 n] staging for positions in caller order
    StepState* st;
    const float* w32;   // 4 * W32Layout::Stride floats
    const void* wfrag;  // 4 * 2 * FragLayout::Count BF16 fragments of 1 KiB (hi, lo)
    const void* wfrag8; // 4 * FragLayout::Count E4M3 fragments of 512 B
    const float* wscale8;  // [4][6] inverse E4M3 weight scales (layers F1 F2 F3 B3 B2 B1)
    // plain- and split-path intermediates (internal atom order)
    float* G;   // [n][384] descriptors
    float* dG;  // [n][384] dE/dG
    // cell lists of large molecules
    const int* molgrid;      // [nmol] grid of the molecule, -1: brute-force candidate scan
    const CellGrid* grids;
    int* cell_count;         // [ncells]
    int* cell_start;         // [ncells + 1]
    int* cell_fill;          // [ncells]
    int* cell_atoms;         // [n]
    int* cellof;             // [n]
};

// Nearest periodic image of a displacement (no-op in the gas phase).  Box
// edges are at least twice the pair-list radius, so the image is unique.
__device__ __forceinline__ void min_image(const Sys& S, double& dx, double& dy, double& dz)
{
    if (S.periodic) {
        dx -= S.box.x * rint(dx * S.ibox.x);
        dy -= S.box.y * rint(dy * S.ibox.y);
        dz -= S.box.z * rint(dz * S.ibox.z);
    }
}

// True when the evaluation that reads this state has to rebuild the pair list.
__device__ __forceinline__ bool rebuild_due(const StepState* st, int rebuild_every)
{
    return !st->lists_valid || st->viol[st->step & 1] || st->age >= rebuild_every;
}

__device__ __forceinline__ int pair_type(int a, int b)
{
    // unordered element pair index: HH HC HN HO CC CN CO NN NO OO
    int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo * 4 - (lo * (lo - 1)) / 2 + (hi - lo);
}

__device__ __forceinline__ float celu_f(float z)
{
    return z > 0.0f ? z : kCeluAlpha * (__expf(z * (1.0f / kCeluAlpha)) - 1.0f);
}

__device__ __forceinline__ float celu_d(float z)
{
    return z > 0.0f ? 1.0f : __expf(z * (1.0f / kCeluAlpha));
}

}  // namespace nnp
