// nnp_api.hip -- host runtime behind the C ABI declared in include/nnp.h.
//
// The context owns the device buffers, the atom permutation between caller
// order and the internal (element, molecule, Morton) order, the stream, and
// the cache of captured HIP graphs for multi-step MD blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/nnp.h"
#include "nnp_internal.h"
#include "nnp_launch.h"

using namespace nnp;

namespace {

constexpr int kShapes[4][2] = {{kH1, kNumFeat}, {kH2, kH1}, {kH3, kH2}, {1, kH3}};
// Molecules with more atoms than this get a cell grid; smaller ones are
// scanned completely by every atom when the pair list is rebuilt.
constexpr int kBruteMax = 4096;
constexpr long long kMaxCellsPerGrid = 1 << 22;
constexpr size_t kBlobPerElement = (size_t)kH1 * kNumFeat + kH1 + (size_t)kH2 * kH1 + kH2 + (size_t)kH3 * kH2 + kH3 + kH3 + 1;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Scratch of the allocation-free stored-mode evaluation
// (nnp_energy_device_static): the descriptors G and dE/dG of at most
// kStaticAtoms atoms, [2][n][384] float, 24 MiB.  Each GPU the library runs
// on holds its own copy until the process ends.  Host code never uses the
// array's name as an address: the per-device address comes from
// hipGetSymbolAddress on the first call on that device (StaticScratch).
constexpr int kStaticAtoms = 8192;
constexpr int kStaticDevices = 64;
static __device__ __align__(256) float scratch[2 * (size_t)kStaticAtoms * kNumFeat];

// Per device: the address of `scratch` on that GPU, and which context's
// G / dE/dG it holds (the last call's; a later call from any context on the
// same GPU replaces them).
struct StaticScratch {
    float* ptr = nullptr;
    const nnp_context* owner = nullptr;
    unsigned long long gen = 0;
};
StaticScratch g_static[kStaticDevices];
std::mutex g_static_mu;

}  // namespace

struct nnp_context {
    std::string err;
    // configuration
    int n = 0, nmol = 0, cap = 160, T = 16;
    int nblk = 4;         // split path: 16-atom column blocks per network workgroup
    bool T_auto = false;  // atoms per tile chosen at layout
    // tiles on the host: table and the atom of every column (kTileCap per tile)
    std::vector<int4> tiles;
    std::vector<int4> tiles_init;  // the table as made (rebalancing reorders tiles)
    std::vector<int> tile_atoms;
    std::vector<int> molgrid;  // grid of each molecule, -1: scanned without a cell grid
    nnp_dtype dtype = NNP_MLP_FP32;
    nnp_path path = NNP_PATH_FUSED;
    bool energy_only = false;  // return_mode NNP_RETURN_ENERGY
    int rebuild_every = 20;
    double skin = 1.0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // caller data
    std::vector<int> species;      // caller order
    std::vector<double> masses;    // caller order
    std::vector<int> mol_of;       // caller order
    std::vector<int> mol_offsets;  // caller order
    std::vector<float> weights;
    // layout (valid once positions were given)
    bool laid_out = false;
    std::vector<int> perm;   // internal -> caller
    std::vector<int> iperm;  // caller -> internal
    // device
    std::vector<DevBuf> bufs;
    Sys S{};
    bool forces_current = false;
    bool kick_pending = false;  // previous block ended after a completed step (mode 1)
    int diff_state = 0;         // 0: none, 1: energy evaluated (recompute), 2: energy + kept G, dE/dG,
                                // 3: as 2 with G, dE/dG in the static scratch (nnp_energy_device_static)
    int static_dev = -1;        // GPU whose static scratch holds this context's G, dE/dG (state 3)
    unsigned long long static_gen = 0;  // that scratch's use count when this context filled it
    // captured MD blocks by (steps, dt, path, dtype, tile, friction, kT, seed)
    std::map<std::tuple<int, double, int, int, int, int, double, double, unsigned long long>, hipGraphExec_t> graphs;
    // extra force providers (caller callbacks and their device buffers)
    struct Extra {
        nnp_force_fn fn;
        void* user;
        double* pos;
        double* frc;
        double* en;
    };
    std::vector<Extra> extra;
    // periodic box (edges, A); all zero in the gas phase
    double box[3] = {0.0, 0.0, 0.0};
    long long cell_cap = 0;  // cells the cell-list arrays hold
    // pinned staging
    double* h_stage = nullptr;
    size_t h_stage_bytes = 0;
    // tile rebalancing: the recorded work read back and the new tile tables
    // uploaded through pinned memory (allocated on first use)
    int* h_work = nullptr;
    int4* h_tiles = nullptr;
    int* h_atoms = nullptr;
    int* h_tmol = nullptr;
    size_t reb_n = 0, reb_nt = 0;  // atoms and tiles these buffers hold
};

namespace {

nnp_status fail(nnp_context* c, nnp_status s, const std::string& msg)
{
    if (c) c->err = msg;
    return s;
}

nnp_status hip_fail(nnp_context* c, hipError_t e, const char* where)
{
    return fail(c, e == hipErrorOutOfMemory ? NNP_ERR_OOM : NNP_ERR_HIP,
                std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
    } while (0)

void* dev_alloc(nnp_context* c, size_t bytes, hipError_t* e)
{
    void* p = nullptr;
    *e = hipMalloc(&p, bytes < 256 ? 256 : bytes);
    if (*e != hipSuccess) return nullptr;
    *e = hipMemset(p, 0, bytes < 256 ? 256 : bytes);
    if (*e != hipSuccess) {
        (void)hipFree(p);
        return nullptr;
    }
    c->bufs.push_back({p, bytes});
    return p;
}

void dev_free(nnp_context* c, const void* p)
{
    for (size_t i = 0; i < c->bufs.size(); ++i)
        if (c->bufs[i].p == p) {
            (void)hipFree(c->bufs[i].p);
            c->bufs.erase(c->bufs.begin() + (long)i);
            return;
        }
}

uint32_t spread_bits(uint32_t v)
{
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000FF;
    v = (v | (v << 8)) & 0x0300F00F;
    v = (v | (v << 4)) & 0x030C30C3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}

// Validates host positions of every molecule: finite, and no two atoms of
// one molecule closer than 1e-6 A (hash on a 1 A grid).
nnp_status check_positions(nnp_context* c, const double* pos)
{
    for (int i = 0; i < 3 * c->n; ++i)
        if (!std::isfinite(pos[i])) return fail(c, NNP_ERR_NONFINITE, "non-finite position component");
    const bool per = c->S.periodic != 0;
    auto coord = [&](int i, int d) {
        const double x = pos[3 * i + d];
        return per ? x - c->box[d] * std::floor(x / c->box[d]) : x;
    };
    std::unordered_map<long long, std::vector<int>> grid;
    for (int m = 0; m < c->nmol; ++m) {
        grid.clear();
        for (int i = c->mol_offsets[m]; i < c->mol_offsets[m + 1]; ++i) {
            const long long gx = (long long)std::floor(coord(i, 0)), gy = (long long)std::floor(coord(i, 1)),
                            gz = (long long)std::floor(coord(i, 2));
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        const long long key = ((gx + dx) * 73856093LL) ^ ((gy + dy) * 19349663LL) ^ ((gz + dz) * 83492791LL);
                        auto it = grid.find(key);
                        if (it == grid.end()) continue;
                        for (int j : it->second) {
                            double ex = pos[3 * i] - pos[3 * j], ey = pos[3 * i + 1] - pos[3 * j + 1],
                                   ez = pos[3 * i + 2] - pos[3 * j + 2];
                            if (per) {
                                ex -= c->box[0] * std::nearbyint(ex / c->box[0]);
                                ey -= c->box[1] * std::nearbyint(ey / c->box[1]);
                                ez -= c->box[2] * std::nearbyint(ez / c->box[2]);
                            }
                            if (ex * ex + ey * ey + ez * ez < 1e-12) {
                                char b[128];
                                snprintf(b, sizeof b, "atoms %d and %d coincide", j, i);
                                return fail(c, NNP_ERR_NONFINITE, b);
                            }
                        }
                    }
            const long long key = (gx * 73856093LL) ^ (gy * 19349663LL) ^ (gz * 83492791LL);
            grid[key].push_back(i);
        }
    }
    return NNP_OK;
}

// Tiles of at most T consecutive atoms of one element (atoms are element-major
// in the internal order).  Workgroups are handed to the eight XCDs round-robin
// (workgroup b runs on XCD b mod 8), so the table is permuted to give each XCD
// one contiguous run of tiles: an XCD then meets one or two elements and its
// L2 holds only their weight fragments.
// Tiles of 16 atoms exceed the LDS of a CU with the FP32 and FP8 networks.
bool fused_tile_ok(int T, nnp_dtype d)
{
    return T == 4 || T == 5 || T == 8 || T == 10 || (T >= 12 && T <= 15) ||
           (T == 16 && (d == NNP_MLP_BF16 || d == NNP_MLP_BF16_SPLIT));
}

// Atoms per descriptor / adjoint workgroup of the split path (8 waves up to
// 7 atoms, 16 waves for 10) and its network's column blocks.
bool split_tile_ok(int T) { return T == 4 || T == 5 || T == 7 || T == 10; }
bool split_dtype_ok(int d) { return d == NNP_MLP_BF16 || d == NNP_MLP_BF16_SPLIT; }

std::vector<int4> make_tiles(const std::vector<int>& elem, int T)
{
    std::vector<int4> seq;
    const int n = (int)elem.size();
    for (int k = 0; k < n;) {
        const int e = elem[k];
        int k2 = k;
        while (k2 < n && elem[k2] == e && k2 - k < T) ++k2;
        seq.push_back(make_int4(k, k2 - k, e, 0));
        k = k2;
    }
    const int nt = (int)seq.size(), q = nt / kXcds, r = nt % kXcds;
    std::vector<int4> out(nt);
    for (int b = 0; b < nt; ++b) {
        const int x = b % kXcds, j = b / kXcds;
        out[b] = seq[x * q + std::min(x, r) + j];
    }
    return out;
}

// Molecule of every tile for the pair-list rebuild shared by a tile's atoms:
// m when all of the tile's atoms belong to molecule m, m is scanned without
// a cell grid and has at most kSharedScanCap atoms, else -1 (each atom then
// scans for itself).  Needed whenever the tiles' atoms or the grids change.
// Synchronous.
// tile_mol entry of every tile (host tables); false before they exist.
bool tile_mol_table(const nnp_context* c, int* tm)
{
    if (c->tiles.empty() || c->molgrid.size() != (size_t)c->nmol || c->perm.size() != (size_t)c->n ||
        c->tile_atoms.size() != c->tiles.size() * kTileCap)
        return false;
    for (size_t b = 0; b < c->tiles.size(); ++b) {
        const int* col = c->tile_atoms.data() + b * kTileCap;
        const int m = c->mol_of[c->perm[col[0]]];
        bool one = c->molgrid[m] < 0 && c->mol_offsets[m + 1] - c->mol_offsets[m] <= kSharedScanCap;
        for (int i = 1; i < c->tiles[b].y && one; ++i) one = c->mol_of[c->perm[col[i]]] == m;
        tm[b] = one ? m : -1;
    }
    return true;
}

nnp_status upload_tile_mol(nnp_context* c)
{
    std::vector<int> tm(c->tiles.size(), -1);
    if (!tile_mol_table(c, tm.data())) return NNP_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy((void*)c->S.tile_mol, tm.data(), sizeof(int) * tm.size(), hipMemcpyHostToDevice));
    return NNP_OK;
}

// Tile table and column atoms (the initial tiling: consecutive atoms) to the
// device.  Synchronous.
nnp_status upload_tiles(nnp_context* c, const std::vector<int4>& tiles)
{
    c->tiles = tiles;
    c->tiles_init = tiles;
    c->tile_atoms.assign(tiles.size() * kTileCap, 0);
    for (size_t b = 0; b < tiles.size(); ++b)
        for (int i = 0; i < tiles[b].y; ++i) c->tile_atoms[b * kTileCap + i] = tiles[b].x + i;
    c->S.ntiles = (int)tiles.size();
    HIP_TRY(c, hipMemcpy((void*)c->S.tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy((void*)c->S.tile_atoms, c->tile_atoms.data(), sizeof(int) * c->tile_atoms.size(),
                         hipMemcpyHostToDevice));
    return upload_tile_mol(c);
}

// Tiles whose atoms pool their angular work take as long as their total
// work.  Between blocks of steps the atoms of each element are
// moved between its tiles, heaviest atom of the heaviest tile for the
// lightest atom of the lightest tile, while that lowers the heavier of the
// two; the work per atom comes from the last evaluation.  Deterministic (a
// function of the recorded work).  Synchronises the context stream.
bool balanced_tiles(const nnp_context* c)
{
    return (c->path == NNP_PATH_FUSED && (c->T == 5 || c->T >= 10)) || c->path == NNP_PATH_SPLIT;
}

void free_rebalance_buffers(nnp_context* c)
{
    if (c->h_work) (void)hipHostFree(c->h_work);
    if (c->h_tiles) (void)hipHostFree(c->h_tiles);
    if (c->h_atoms) (void)hipHostFree(c->h_atoms);
    if (c->h_tmol) (void)hipHostFree(c->h_tmol);
    c->h_work = c->h_atoms = c->h_tmol = nullptr;
    c->h_tiles = nullptr;
    c->reb_n = c->reb_nt = 0;
}

// The device stays idle while the tiles are rebalanced between blocks, so
// the read-back and the uploads go through pinned buffers, and the uploads
// are left in flight: the graph launch that follows is ordered after them,
// and the next rebalancing synchronises the stream before it rewrites the
// buffers.
nnp_status rebalance_tiles(nnp_context* c)
{
    if (!balanced_tiles(c) || !c->laid_out) return NNP_OK;
    const int n = c->n, nt = (int)c->tiles.size();
    if (c->reb_n != (size_t)n || c->reb_nt != (size_t)nt) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        free_rebalance_buffers(c);
        HIP_TRY(c, hipHostMalloc((void**)&c->h_work, sizeof(int) * n));
        HIP_TRY(c, hipHostMalloc((void**)&c->h_tiles, sizeof(int4) * nt));
        HIP_TRY(c, hipHostMalloc((void**)&c->h_atoms, sizeof(int) * nt * kTileCap));
        HIP_TRY(c, hipHostMalloc((void**)&c->h_tmol, sizeof(int) * nt));
        c->reb_n = n;
        c->reb_nt = nt;
    }
    int* work = c->h_work;
    HIP_TRY(c, hipMemcpyAsync(work, c->S.work, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    bool changed = false;
    for (int e = 0; e < kNumSpecies; ++e) {
        std::vector<int> tl;
        for (int b = 0; b < nt; ++b)
            if (c->tiles[b].z == e) tl.push_back(b);
        if (tl.size() < 2) continue;
        std::vector<long long> W(nt, 0);
        for (int b : tl)
            for (int i = 0; i < c->tiles[b].y; ++i) W[b] += work[c->tile_atoms[b * kTileCap + i]];
        for (size_t it = 0; it < 8 * tl.size(); ++it) {
            int h = tl[0], l = tl[0];
            for (int b : tl) {
                if (W[b] > W[h]) h = b;
                if (W[b] < W[l]) l = b;
            }
            if (h == l) break;
            int ih = 0, il = 0;
            for (int i = 1; i < c->tiles[h].y; ++i)
                if (work[c->tile_atoms[h * kTileCap + i]] > work[c->tile_atoms[h * kTileCap + ih]]) ih = i;
            for (int i = 1; i < c->tiles[l].y; ++i)
                if (work[c->tile_atoms[l * kTileCap + i]] < work[c->tile_atoms[l * kTileCap + il]]) il = i;
            const int ah = c->tile_atoms[h * kTileCap + ih], al = c->tile_atoms[l * kTileCap + il];
            const long long d = (long long)work[ah] - work[al];
            if (d <= 0 || std::max(W[h] - d, W[l] + d) >= W[h]) break;
            std::swap(c->tile_atoms[h * kTileCap + ih], c->tile_atoms[l * kTileCap + il]);
            W[h] -= d;
            W[l] += d;
            changed = true;
        }
    }
    // Schedule: workgroups start in index order and workgroup b runs on die
    // b mod 8, so each die's entries (b = x, x + 8, ...) are reordered by
    // their tiles' recorded work, heaviest first: long tiles start first and
    // short ones fill the end of the launch (list scheduling by work).  A
    // device-side queue (an atomic counter per die) gave the same order at
    // the price of a contended atomic and a dependent load before every
    // tile's first access; this order costs nothing on the device.
    {
        std::vector<long long> W(nt, 0);
        for (int b = 0; b < nt; ++b)
            for (int i = 0; i < c->tiles[b].y; ++i) W[b] += work[c->tile_atoms[(size_t)b * kTileCap + i]];
        std::vector<int4> tiles2(c->tiles);
        std::vector<int> atoms2(c->tile_atoms);
        for (int x = 0; x < kXcds; ++x) {
            std::vector<int> idx;
            for (int b = x; b < nt; b += kXcds) idx.push_back(b);
            std::vector<int> srt(idx);
            std::stable_sort(srt.begin(), srt.end(), [&](int p, int q) { return W[p] > W[q]; });
            for (size_t k = 0; k < idx.size(); ++k) {
                if (srt[k] == idx[k]) continue;
                tiles2[idx[k]] = c->tiles[srt[k]];
                std::copy(c->tile_atoms.begin() + (size_t)srt[k] * kTileCap,
                          c->tile_atoms.begin() + (size_t)(srt[k] + 1) * kTileCap,
                          atoms2.begin() + (size_t)idx[k] * kTileCap);
                changed = true;
            }
        }
        c->tiles.swap(tiles2);
        c->tile_atoms.swap(atoms2);
    }
    if (changed) {
        std::copy(c->tiles.begin(), c->tiles.end(), c->h_tiles);
        std::copy(c->tile_atoms.begin(), c->tile_atoms.end(), c->h_atoms);
        HIP_TRY(c, hipMemcpyAsync((void*)c->S.tiles, c->h_tiles, sizeof(int4) * nt, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync((void*)c->S.tile_atoms, c->h_atoms, sizeof(int) * (size_t)nt * kTileCap,
                                  hipMemcpyHostToDevice, c->stream));
        if (tile_mol_table(c, c->h_tmol))
            HIP_TRY(c, hipMemcpyAsync((void*)c->S.tile_mol, c->h_tmol, sizeof(int) * nt, hipMemcpyHostToDevice,
                                      c->stream));
    }
    return NNP_OK;
}

// Cell grids of the molecules with more than kBruteMax atoms (the others scan
// every atom of their molecule).  Gas phase: a grid around the molecule's
// positions `pos` (caller order) with margins; periodic box: the box itself
// split into floor(L / (5.2 + skin)) cells per edge when that is at least 3
// in every dimension (else the scan with nearest images).
nnp_status setup_grids(nnp_context* c, const double* pos)
{
    Sys& S = c->S;
    // the grid arrays below are rewritten from the host: nothing of this
    // context may still be reading them
    if (c->stream) HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<int> molgrid(c->nmol, -1);
    std::vector<CellGrid> grids;
    long long ncells = 0;
    const double rl = 5.2 + c->skin;
    for (int m = 0; m < c->nmol; ++m) {
        const int lo = c->mol_offsets[m], hi = c->mol_offsets[m + 1];
        if (hi - lo <= kBruteMax) continue;
        CellGrid G{};
        int nd[3];
        if (S.periodic) {
            long long cells = 1;
            for (int d = 0; d < 3; ++d) {
                nd[d] = (int)std::min<double>(std::floor(c->box[d] / rl), 1024.0);
                cells *= nd[d];
            }
            if (nd[0] < 3 || nd[1] < 3 || nd[2] < 3) continue;
            while (cells > kMaxCellsPerGrid) {
                cells = 1;
                for (int d = 0; d < 3; ++d) {
                    nd[d] = std::max(3, (nd[d] * 4) / 5);
                    cells *= nd[d];
                }
            }
            G.ox = G.oy = G.oz = 0.0;
            G.ihx = nd[0] / c->box[0];
            G.ihy = nd[1] / c->box[1];
            G.ihz = nd[2] / c->box[2];
            G.periodic = 1;
        } else {
            double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
            for (int i = lo; i < hi; ++i)
                for (int d = 0; d < 3; ++d) {
                    mn[d] = std::min(mn[d], pos[3 * i + d]);
                    mx[d] = std::max(mx[d], pos[3 * i + d]);
                }
            double org[3], span[3];
            for (int d = 0; d < 3; ++d) {
                const double L = mx[d] - mn[d];
                const double margin = std::max(2.0 * rl, 0.5 * L);
                org[d] = mn[d] - margin;
                span[d] = L + 2.0 * margin;
            }
            double h = rl;
            for (;;) {
                long long cells = 1;
                for (int d = 0; d < 3; ++d) {
                    nd[d] = std::max(1, (int)std::ceil(span[d] / h));
                    cells *= nd[d];
                }
                if (cells <= kMaxCellsPerGrid) break;
                h *= 1.25;
            }
            G.ox = org[0];
            G.oy = org[1];
            G.oz = org[2];
            G.ihx = G.ihy = G.ihz = 1.0 / h;
            G.periodic = 0;
        }
        G.nx = nd[0];
        G.ny = nd[1];
        G.nz = nd[2];
        G.first = (int)ncells;
        ncells += (long long)nd[0] * nd[1] * nd[2];
        molgrid[m] = (int)grids.size();
        grids.push_back(G);
    }
    HIP_TRY(c, hipMemcpy((void*)S.molgrid, molgrid.data(), sizeof(int) * c->nmol, hipMemcpyHostToDevice));
    if (ncells > c->cell_cap) {
        dev_free(c, S.grids);
        dev_free(c, S.cell_count);
        dev_free(c, S.cell_start);
        dev_free(c, S.cell_fill);
        hipError_t e = hipSuccess;
        S.grids = (const CellGrid*)dev_alloc(c, sizeof(CellGrid) * c->nmol, &e);
        if (e == hipSuccess) S.cell_count = (int*)dev_alloc(c, sizeof(int) * ncells, &e);
        if (e == hipSuccess) S.cell_start = (int*)dev_alloc(c, sizeof(int) * (ncells + 1), &e);
        if (e == hipSuccess) S.cell_fill = (int*)dev_alloc(c, sizeof(int) * ncells, &e);
        if (e == hipSuccess && !S.cell_atoms) S.cell_atoms = (int*)dev_alloc(c, sizeof(int) * c->n, &e);
        if (e == hipSuccess && !S.cellof) S.cellof = (int*)dev_alloc(c, sizeof(int) * c->n, &e);
        if (e != hipSuccess) return hip_fail(c, e, "cell list allocation");
        c->cell_cap = ncells;
    }
    S.ncells = (int)ncells;
    if (ncells > 0) {
        HIP_TRY(c, hipMemcpy((void*)S.grids, grids.data(), sizeof(CellGrid) * grids.size(), hipMemcpyHostToDevice));
        // the cell scan clears what it reads; a new layout starts from zero
        HIP_TRY(c, hipMemset(S.cell_count, 0, sizeof(int) * ncells));
        HIP_TRY(c, hipMemset(S.cell_fill, 0, sizeof(int) * ncells));
    }
    c->molgrid = molgrid;
    return upload_tile_mol(c);
}

// Network tiles of the split path: up to 16 nblk consecutive atoms of one
// element, in the same die-contiguous order as the tiles.  Synchronous.
nnp_status upload_wide_tiles(nnp_context* c, const std::vector<int>& elem)
{
    if (c->path != NNP_PATH_SPLIT || !c->S.wtiles) return NNP_OK;
    const std::vector<int4> wt = make_tiles(elem, 16 * c->nblk);
    c->S.nwtiles = (int)wt.size();
    c->S.wide_blk = c->nblk;
    HIP_TRY(c, hipMemcpy((void*)c->S.wtiles, wt.data(), sizeof(int4) * wt.size(), hipMemcpyHostToDevice));
    return NNP_OK;
}

// Builds the internal order from the first positions and uploads every
// per-atom constant.
nnp_status lay_out(nnp_context* c, const double* pos)
{
    const int n = c->n;
    std::vector<uint64_t> key(n);
    for (int m = 0; m < c->nmol; ++m) {
        const int lo = c->mol_offsets[m], hi = c->mol_offsets[m + 1];
        double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
        auto coord = [&](int i, int d) {
            const double x = pos[3 * i + d];
            return c->S.periodic ? x - c->box[d] * std::floor(x / c->box[d]) : x;
        };
        for (int i = lo; i < hi; ++i)
            for (int d = 0; d < 3; ++d) {
                mn[d] = std::min(mn[d], coord(i, d));
                mx[d] = std::max(mx[d], coord(i, d));
            }
        for (int i = lo; i < hi; ++i) {
            uint32_t q[3];
            for (int d = 0; d < 3; ++d) {
                const double span = std::max(mx[d] - mn[d], 1e-9);
                q[d] = (uint32_t)std::min(1023.0, std::max(0.0, std::floor((coord(i, d) - mn[d]) / span * 1023.999)));
            }
            const uint64_t morton = spread_bits(q[0]) | (spread_bits(q[1]) << 1) | (spread_bits(q[2]) << 2);
            key[i] = ((uint64_t)c->species[i] << 60) | ((uint64_t)m << 32) | morton;
        }
    }
    c->perm.resize(n);
    std::iota(c->perm.begin(), c->perm.end(), 0);
    std::stable_sort(c->perm.begin(), c->perm.end(), [&](int a, int b) { return key[a] < key[b]; });
    c->iperm.assign(n, 0);
    for (int k = 0; k < n; ++k) c->iperm[c->perm[k]] = k;

    // per-atom constants in internal order
    std::vector<double4> p4(n);
    std::vector<double> kinv(n), mass(n);
    std::vector<int> mol(n);
    for (int k = 0; k < n; ++k) {
        const int i = c->perm[k];
        p4[k] = make_double4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], (double)c->species[i]);
        mass[k] = c->masses[i];
        kinv[k] = kKappa / c->masses[i];
        mol[k] = c->mol_of[i];
    }
    // molecule x element ranges
    std::vector<int2> mr((size_t)c->nmol * 4, make_int2(0, 0));
    for (int k = 0; k < n;) {
        const int m = mol[k], e = (int)p4[k].w;
        int k2 = k;
        while (k2 < n && mol[k2] == m && (int)p4[k2].w == e) ++k2;
        mr[(size_t)m * 4 + e] = make_int2(k, k2);
        k = k2;
    }
    std::vector<int> elem(n);
    for (int k = 0; k < n; ++k) elem[k] = (int)p4[k].w;
    if (c->T_auto) {
        // the smallest of 8, 10, 12-15 (and 16 with the BF16 networks) atoms
        // per tile that gives one workgroup per CU (a second one on a CU runs
        // after the first); for more tiles than CUs the pooled tile size with
        // the least time in rounds of one tile per CU, a tile taking ~21 us +
        // ~1 us per atom (per-workgroup stamps of the 10-14-atom kernels)
        const int Tmax = fused_tile_ok(16, c->dtype) ? 16 : 15;
        int dev = 0, ncu = 256;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        c->T = 0;
        for (int T : {8, 10, 12, 13, 14, 15, 16})
            if (T <= Tmax && make_tiles(elem, T).size() <= (size_t)ncu) {
                c->T = T;
                break;
            }
        if (c->T == 0) {
            double best = 0.0;
            for (int T : {10, 12, 13, 14, 15, 16}) {
                if (T > Tmax) break;
                const double rounds = (double)((make_tiles(elem, T).size() + ncu - 1) / ncu);
                const double cost = rounds * (21.0 + T);
                if (c->T == 0 || cost < best) {
                    best = cost;
                    c->T = T;
                }
            }
        }
    }
    const std::vector<int4> tiles = make_tiles(elem, c->T);
    std::vector<int> perm_dev(c->perm.begin(), c->perm.end());
    Sys& S = c->S;
    S.ntiles = (int)tiles.size();
    {
        const nnp_status gs = setup_grids(c, pos);
        if (gs != NNP_OK) return gs;
    }
    HIP_TRY(c, hipMemcpy(S.pos, p4.data(), sizeof(double4) * n, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy((void*)S.kinv, kinv.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy((void*)S.mass, mass.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy((void*)S.mol, mol.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy((void*)S.mrange, mr.data(), sizeof(int2) * mr.size(), hipMemcpyHostToDevice));
    {
        const nnp_status ts = upload_tiles(c, tiles);
        if (ts != NNP_OK) return ts;
        const nnp_status ws = upload_wide_tiles(c, elem);
        if (ws != NNP_OK) return ws;
    }
    HIP_TRY(c, hipMemcpy((void*)S.perm, perm_dev.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    // the context stream does not synchronise with the null stream
    HIP_TRY(c, hipDeviceSynchronize());
    c->laid_out = true;
    return NNP_OK;
}

// Buffers of the split path (G, dE/dG, network tiles), allocated on first use.
nnp_status split_buffers(nnp_context* c)
{
    hipError_t e = hipSuccess;
    Sys& S = c->S;
    if (!S.G) S.G = (float*)dev_alloc(c, sizeof(float) * (size_t)c->n * kNumFeat, &e);
    if (e == hipSuccess && !S.dG) S.dG = (float*)dev_alloc(c, sizeof(float) * (size_t)c->n * kNumFeat, &e);
    if (e == hipSuccess && !S.wtiles) S.wtiles = (const int4*)dev_alloc(c, sizeof(int4) * ((size_t)c->n / 16 + 8), &e);
    if (e != hipSuccess) return hip_fail(c, e, "split-path buffers");
    return NNP_OK;
}

// Rebuilds the tile tables for a new path / atoms-per-tile / network tile.
nnp_status retile(nnp_context* c, int T, nnp_path path, int nblk)
{
    if (path == NNP_PATH_SPLIT) {
        const nnp_status bs = split_buffers(c);
        if (bs != NNP_OK) return bs;
    }
    c->T = T;
    c->path = path;
    c->nblk = nblk;
    if (!c->laid_out) return NNP_OK;
    std::vector<int> elem(c->n);
    for (int k = 0; k < c->n; ++k) elem[k] = c->species[c->perm[k]];
    const std::vector<int4> tiles = make_tiles(elem, T);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    nnp_status ts = upload_tiles(c, tiles);
    if (ts == NNP_OK) ts = upload_wide_tiles(c, elem);
    if (ts != NNP_OK) return ts;
    HIP_TRY(c, hipDeviceSynchronize());
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
    return NNP_OK;
}

// OCP FP8 E4M3 (bias 7, no infinities, 0x7f/0xff NaN, largest finite 448):
// round to nearest even, values beyond 448 saturate to 448.
uint8_t e4m3_encode(float x)
{
    const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
    const float a = std::fabs(x);
    if (std::isnan(a)) return 0x7f;
    if (a >= 448.0f) return sign | 0x7e;
    if (a < std::ldexp(1.0f, -6)) {  // subnormal: m * 2^-9, m = 0..7 (8 is the smallest normal)
        const int m = (int)std::nearbyint(a * 512.0f);
        return sign | (uint8_t)m;
    }
    int e2;
    std::frexp(a, &e2);
    int E = e2 - 1;  // a = (1 + m/8) 2^E
    int m = (int)std::nearbyint((a / std::ldexp(1.0f, E) - 1.0f) * 8.0f);
    if (m == 8) {
        m = 0;
        ++E;
    }
    int code = ((E + 7) << 3) | m;
    if (code > 0x7e) code = 0x7e;
    return sign | (uint8_t)code;
}

void build_weights(const std::vector<float>& blob, std::vector<float>& w32, std::vector<uint16_t>& frag,
                   std::vector<uint8_t>& frag8, std::vector<float>& wscale8)
{
    frag8.assign((size_t)4 * FragLayout::Count * 512, 0);
    wscale8.assign(4 * 6, 1.0f);
    w32.assign((size_t)4 * W32Layout::Stride, 0.f);
    frag.assign((size_t)4 * 2 * FragLayout::Count * 64 * 8, 0);
    auto bf16 = [](float x) -> uint16_t {  // round to nearest even
        uint32_t u;
        std::memcpy(&u, &x, 4);
        if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    };
    for (int e = 0; e < 4; ++e) {
        const float* p = blob.data() + (size_t)e * kBlobPerElement;
        const float* W[4];
        const float* b[4];
        size_t off = 0;
        for (int l = 0; l < 4; ++l) {
            W[l] = p + off;
            off += (size_t)kShapes[l][0] * kShapes[l][1];
            b[l] = p + off;
            off += kShapes[l][0];
        }
        float* o = w32.data() + (size_t)e * W32Layout::Stride;
        auto put_t = [&](int dst, const float* Wm, int M, int K) {  // [K][M] = W^T
            for (int k = 0; k < K; ++k)
                for (int m = 0; m < M; ++m) o[dst + k * M + m] = Wm[(size_t)m * K + k];
        };
        auto put = [&](int dst, const float* Wm, int M, int K) {
            std::memcpy(o + dst, Wm, sizeof(float) * M * K);
        };
        put_t(W32Layout::Wt1, W[0], kH1, kNumFeat);
        put(W32Layout::W1, W[0], kH1, kNumFeat);
        put_t(W32Layout::Wt2, W[1], kH2, kH1);
        put(W32Layout::W2, W[1], kH2, kH1);
        put_t(W32Layout::Wt3, W[2], kH3, kH2);
        put(W32Layout::W3, W[2], kH3, kH2);
        std::memcpy(o + W32Layout::W4, W[3], sizeof(float) * kH3);
        std::memcpy(o + W32Layout::B1, b[0], sizeof(float) * kH1);
        std::memcpy(o + W32Layout::B2, b[1], sizeof(float) * kH2);
        std::memcpy(o + W32Layout::B3, b[2], sizeof(float) * kH3);
        o[W32Layout::B4] = b[3][0];
        // MFMA A fragments: fragment (mt, kt), lane l, value i holds
        // A[16 mt + l % 16][32 kt + 8 (l / 16) + i]
        // hi fragments, then lo = bf16(w - hi) fragments of the same layout
        uint16_t* fr = frag.data() + (size_t)e * 2 * FragLayout::Count * 512;
        uint16_t* frl = fr + (size_t)FragLayout::Count * 512;
        auto put_frag = [&](int base, int M, int K, bool transpose, const float* Wm, int ldw) {
            const int KT = K / 32;
            for (int mt = 0; mt < M / 16; ++mt)
                for (int kt = 0; kt < KT; ++kt)
                    for (int l = 0; l < 64; ++l)
                        for (int i = 0; i < 8; ++i) {
                            const int r = 16 * mt + (l % 16), k = 32 * kt + 8 * (l / 16) + i;
                            const float v = transpose ? Wm[(size_t)k * ldw + r] : Wm[(size_t)r * ldw + k];
                            const size_t at = ((size_t)(base + mt * KT + kt) * 64 + l) * 8 + i;
                            const uint16_t h = bf16(v);
                            uint32_t hb = (uint32_t)h << 16;
                            float hf;
                            std::memcpy(&hf, &hb, 4);
                            fr[at] = h;
                            frl[at] = bf16(v - hf);
                        }
        };
        put_frag(FragLayout::F1, kH1, kNumFeat, false, W[0], kNumFeat);
        put_frag(FragLayout::F2, kH2, kH1, false, W[1], kH1);
        put_frag(FragLayout::F3, kH3, kH2, false, W[2], kH2);
        put_frag(FragLayout::B3, kH2, kH3, true, W[2], kH2);
        put_frag(FragLayout::B2, kH1, kH2, true, W[1], kH1);
        put_frag(FragLayout::B1, kNumFeat, kH1, true, W[0], kNumFeat);
        // E4M3 fragments, one static scale 448 / amax|W| per matrix
        uint8_t* f8 = frag8.data() + (size_t)e * FragLayout::Count * 512;
        auto put_frag8 = [&](int layer, int base, int M, int K, bool transpose, const float* Wm, int ldw, int nW) {
            float amax = 0.f;
            for (int i = 0; i < nW; ++i) amax = std::max(amax, std::fabs(Wm[i]));
            const float sc = amax > 0.f ? 448.0f / amax : 1.0f;
            wscale8[e * 6 + layer] = 1.0f / sc;
            const int KT = K / 32;
            for (int mt = 0; mt < M / 16; ++mt)
                for (int kt = 0; kt < KT; ++kt)
                    for (int l = 0; l < 64; ++l)
                        for (int i = 0; i < 8; ++i) {
                            const int r = 16 * mt + (l % 16), k = 32 * kt + 8 * (l / 16) + i;
                            const float v = transpose ? Wm[(size_t)k * ldw + r] : Wm[(size_t)r * ldw + k];
                            f8[((size_t)(base + mt * KT + kt) * 64 + l) * 8 + i] = e4m3_encode(v * sc);
                        }
        };
        put_frag8(0, FragLayout::F1, kH1, kNumFeat, false, W[0], kNumFeat, kH1 * kNumFeat);
        put_frag8(1, FragLayout::F2, kH2, kH1, false, W[1], kH1, kH2 * kH1);
        put_frag8(2, FragLayout::F3, kH3, kH2, false, W[2], kH2, kH3 * kH2);
        put_frag8(3, FragLayout::B3, kH2, kH3, true, W[2], kH2, kH3 * kH2);
        put_frag8(4, FragLayout::B2, kH1, kH2, true, W[1], kH1, kH2 * kH1);
        put_frag8(5, FragLayout::B1, kNumFeat, kH1, true, W[0], kNumFeat, kH1 * kNumFeat);
    }
}

int mode_of(const nnp_context* c)
{
    switch (c->dtype) {
        case NNP_MLP_BF16: return 1;
        case NNP_MLP_BF16_SPLIT: return 2;
        case NNP_MLP_FP8: return 3;
        default: return 0;
    }
}

hipError_t enqueue_eval(nnp_context* c, bool grad)
{
    return launch_eval(c->S, (int)c->path, mode_of(c), c->T, grad, c->stream);
}

// Evaluation at the current positions without integration (forces, energies).
hipError_t enqueue_compute(nnp_context* c, bool grad)
{
    hipError_t e = enqueue_eval(c, grad);
    if (e != hipSuccess) return e;
    if (!grad) {
        // energy-only: per-slot forces are not written; the gather would read
        // stale slots, so zero-force semantics are not provided -- only the
        // energies of this evaluation are meaningful
    }
    return launch_gather_integrate(c->S, 0.0, 0, c->stream);
}

// Runs the extra force providers on the evaluation just enqueued: each gets
// the positions, adds its forces and energies, and the library adds them to
// the evaluation's sums before the gather.
nnp_status apply_extra(nnp_context* c)
{
    for (size_t k = 0; k < c->extra.size(); ++k) {
        const auto& x = c->extra[k];
        HIP_TRY(c, launch_extra_prepare(c->S, x.pos, x.frc, x.en, c->stream));
        const int rc = x.fn(x.user, c->n, c->nmol, x.pos, x.frc, x.en, (void*)c->stream);
        if (rc != 0) {
            // the evaluation is discarded: a gather without integration empties
            // its force and energy sums so that the next evaluation starts clean
            (void)launch_gather_integrate(c->S, 0.0, 0, c->stream);
            (void)hipStreamSynchronize(c->stream);
            c->forces_current = false;
            c->kick_pending = false;
            char b[96];
            snprintf(b, sizeof b, "force provider %d returned %d", (int)k, rc);
            return fail(c, NNP_ERR_STATE, b);
        }
        HIP_TRY(c, launch_extra_add(c->S, x.frc, x.en, c->stream));
    }
    return NNP_OK;
}

// One complete evaluation: network energies (and forces when grad), extra
// providers, force gather.  Without grad the network's forward runs alone
// and the gather leaves the context's forces untouched (it still empties the
// fixed-point sums that the providers may have filled).
nnp_status full_compute(nnp_context* c, bool grad = true)
{
    HIP_TRY(c, enqueue_eval(c, grad));
    const nnp_status xs = apply_extra(c);
    if (xs != NNP_OK) return xs;
    HIP_TRY(c, launch_gather_integrate(c->S, 0.0, 0, c->stream, grad));
    return NNP_OK;
}

// Steps with extra providers: launched one by one (the providers are host
// code, so the steps are not captured in graphs).
nnp_status steps_with_extra(nnp_context* c, double dt, int nsteps)
{
    HIP_TRY(c, launch_kickdrift(c->S, dt, c->stream));
    for (int i = 0; i < nsteps; ++i) {
        HIP_TRY(c, enqueue_eval(c, true));
        const nnp_status xs = apply_extra(c);
        if (xs != NNP_OK) return xs;
        HIP_TRY(c, launch_gather_integrate(c->S, dt, i == nsteps - 1 ? 1 : 2, c->stream));
    }
    return NNP_OK;
}

hipError_t enqueue_steps(nnp_context* c, double dt, int nsteps, bool first_kick)
{
    hipError_t e = hipSuccess;
    if (first_kick) e = launch_kickdrift(c->S, dt, c->stream);
    for (int i = 0; i < nsteps && e == hipSuccess; ++i) {
        e = enqueue_eval(c, true);
        if (e == hipSuccess) e = launch_gather_integrate(c->S, dt, i == nsteps - 1 ? 1 : 2, c->stream);
    }
    return e;
}

// Steps per captured block of nnp_step.  Each block boundary costs a host
// synchronisation, the tile rebalancing from the recorded work and a graph
// launch (~0.2 ms with the GPU idle at 2,500 atoms); 200 steps per block
// halve that cost against 100 (+2 % MD steps/s at 2,500 atoms) without a
// measurable loss of balance, and 250 gained nothing more.
constexpr int kGraphBlock = 200;

// The executable graph of one block of len steps (captured and instantiated
// on first use, then cached by everything its kernel arguments depend on).
nnp_status block_graph(nnp_context* c, double dt, int len, hipGraphExec_t* out)
{
    const auto key = std::make_tuple(len, dt, (int)c->path, (int)c->dtype, c->T, c->nblk, c->S.gamma, c->S.kT,
                                     c->S.seed);
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        hipGraph_t g;
        HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_steps(c, dt, len, true);
        hipError_t e2 = hipStreamEndCapture(c->stream, &g);
        if (e != hipSuccess) return hip_fail(c, e, "capture");
        if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
        hipGraphExec_t x;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
        it = c->graphs.emplace(key, x).first;
    }
    *out = it->second;
    return NNP_OK;
}

nnp_status check_device_flags(nnp_context* c)
{
    StepState st;
    HIP_TRY(c, hipMemcpyAsync(&st, c->S.st, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (st.overflow) {
        char b[256];
        snprintf(b, sizeof b,
                 "capacity exceeded: largest pair list %d (max_neighbors %d), neighbours within 5.2 A %d (max %d), "
                 "within 3.5 A %d (max %d)",
                 st.max_ns, c->cap, st.max_nr, kRadMax, st.max_na, kAngMax);
        return fail(c, NNP_ERR_STATE, b);
    }
    if (st.nonfinite) return fail(c, NNP_ERR_NONFINITE, "non-finite energy or force on the device");
    return NNP_OK;
}

nnp_status upload_positions(nnp_context* c, const double* pos)
{
    nnp_status s = check_positions(c, pos);
    if (s != NNP_OK) return s;
    if (!c->laid_out) return lay_out(c, pos);
    HIP_TRY(c, hipMemcpyAsync(c->S.stage, pos, sizeof(double) * 3 * c->n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, launch_positions_in(c->S, c->S.stage, 1, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return NNP_OK;
}

}  // namespace

extern "C" {

const char* nnp_status_string(nnp_status s)
{
    switch (s) {
        case NNP_OK: return "NNP_OK";
        case NNP_ERR_ARG: return "NNP_ERR_ARG";
        case NNP_ERR_NONFINITE: return "NNP_ERR_NONFINITE";
        case NNP_ERR_UNSUPPORTED: return "NNP_ERR_UNSUPPORTED";
        case NNP_ERR_OOM: return "NNP_ERR_OOM";
        case NNP_ERR_HIP: return "NNP_ERR_HIP";
        case NNP_ERR_STATE: return "NNP_ERR_STATE";
    }
    return "NNP_ERR_UNKNOWN";
}

const char* nnp_last_error(const nnp_context* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// An enum field of the caller's struct as the integer it holds: a C caller
// may store any int there, and reading a value outside the enumerators
// through the C++ enum type is undefined.
static int enum_raw(const void* field)
{
    int v;
    std::memcpy(&v, field, sizeof v);
    return v;
}

static nnp_status validate_params(const nnp_params* p, std::string& msg)
{
    if (!p) return msg = "params is NULL", NNP_ERR_ARG;
    if (p->n_atoms <= 0) return msg = "n_atoms must be > 0", NNP_ERR_ARG;
    if (p->n_molecules < 1 || p->n_molecules > p->n_atoms) return msg = "n_molecules out of range", NNP_ERR_ARG;
    if (p->n_molecules > 1 && !p->mol_offsets) return msg = "mol_offsets is NULL", NNP_ERR_ARG;
    if (p->mol_offsets) {
        if (p->mol_offsets[0] != 0 || p->mol_offsets[p->n_molecules] != p->n_atoms)
            return msg = "mol_offsets must start at 0 and end at n_atoms", NNP_ERR_ARG;
        for (int m = 0; m < p->n_molecules; ++m)
            if (p->mol_offsets[m + 1] <= p->mol_offsets[m]) return msg = "empty or decreasing molecule", NNP_ERR_ARG;
    }
    if (!p->species || !p->masses || !p->weights) return msg = "species, masses and weights are required", NNP_ERR_ARG;
    for (int i = 0; i < p->n_atoms; ++i) {
        if (p->species[i] < 0 || p->species[i] > 3) return msg = "species outside {0,1,2,3}", NNP_ERR_ARG;
        if (!(p->masses[i] > 0.0) || !std::isfinite(p->masses[i])) return msg = "mass must be finite and > 0", NNP_ERR_ARG;
    }
    if (p->weights_count != 4 * kBlobPerElement) return msg = "weights_count must be 4 * 94689", NNP_ERR_ARG;
    for (size_t i = 0; i < p->weights_count; ++i)
        if (!std::isfinite(p->weights[i])) return msg = "non-finite weight", NNP_ERR_NONFINITE;
    static_assert(sizeof(nnp_dtype) == sizeof(int) && sizeof(nnp_path) == sizeof(int) &&
                      sizeof(nnp_return) == sizeof(int),
                  "enum fields are int-sized");
    const int dt = enum_raw(&p->mlp_dtype), pa = enum_raw(&p->path), rm = enum_raw(&p->return_mode);
    if (dt != NNP_MLP_FP32 && dt != NNP_MLP_BF16 && dt != NNP_MLP_BF16_SPLIT && dt != NNP_MLP_FP8)
        return msg = "unknown mlp_dtype", NNP_ERR_ARG;
    if (pa != NNP_PATH_PLAIN && pa != NNP_PATH_FUSED && pa != NNP_PATH_SPLIT) return msg = "unknown path", NNP_ERR_ARG;
    if (pa == NNP_PATH_SPLIT && !split_dtype_ok(dt))
        return msg = "the split path runs the BF16 and split-BF16 networks only", NNP_ERR_UNSUPPORTED;
    if (rm != 0 && rm != NNP_RETURN_ENERGY && rm != NNP_RETURN_ENERGY_FORCES)
        return msg = "unknown return_mode", NNP_ERR_ARG;
    if (p->rebuild_every < 1) return msg = "rebuild_every must be >= 1", NNP_ERR_ARG;
    if (!(p->skin >= 0.0) || !std::isfinite(p->skin) || p->skin > 5.0) return msg = "skin must be in [0, 5] A", NNP_ERR_ARG;
    if (p->max_neighbors < 0 || p->max_neighbors > kCapMax) return msg = "max_neighbors must be in [0, 256]", NNP_ERR_ARG;
    if (p->path == NNP_PATH_FUSED && p->atoms_per_tile != 0 && !fused_tile_ok(p->atoms_per_tile, p->mlp_dtype))
        return msg = "atoms_per_tile of the fused path must be 0, 4, 5, 8, 10, 12-15 or (BF16 networks) 16", NNP_ERR_ARG;
    if (p->path == NNP_PATH_PLAIN && p->atoms_per_tile != 0 && p->atoms_per_tile != 8 && p->atoms_per_tile != 16)
        return msg = "atoms_per_tile of the plain path must be 0, 8 or 16", NNP_ERR_ARG;
    if (p->path == NNP_PATH_SPLIT && p->atoms_per_tile != 0 && !split_tile_ok(p->atoms_per_tile))
        return msg = "atoms_per_tile of the split path must be 0, 4, 5, 7 or 10", NNP_ERR_ARG;
    if (p->network_tile != 0 && p->network_tile != 16 && p->network_tile != 32 && p->network_tile != 48 &&
        p->network_tile != 64)
        return msg = "network_tile must be 0, 16, 32, 48 or 64", NNP_ERR_ARG;
    return NNP_OK;
}

nnp_status nnp_create(const nnp_params* p, nnp_context** out)
{
    if (!out) return NNP_ERR_ARG;
    *out = nullptr;
    std::string msg;
    nnp_status s = validate_params(p, msg);
    if (s != NNP_OK) {
        fprintf(stderr, "nnp_create: %s\n", msg.c_str());
        return s;
    }
    nnp_context* c = new (std::nothrow) nnp_context();
    if (!c) return NNP_ERR_OOM;
    c->n = p->n_atoms;
    c->nmol = p->n_molecules;
    c->cap = p->max_neighbors ? p->max_neighbors : 192;
    c->T = p->atoms_per_tile ? p->atoms_per_tile
                             : (p->path == NNP_PATH_FUSED ? 8 : p->path == NNP_PATH_SPLIT ? 5 : 16);
    c->nblk = p->network_tile ? p->network_tile / 16 : 4;
    c->T_auto = p->atoms_per_tile == 0 && p->path == NNP_PATH_FUSED;
    c->dtype = p->mlp_dtype;
    c->path = p->path;
    c->energy_only = p->return_mode == NNP_RETURN_ENERGY;
    c->rebuild_every = p->rebuild_every;
    c->skin = p->skin;
    c->species.assign(p->species, p->species + c->n);
    c->masses.assign(p->masses, p->masses + c->n);
    c->weights.assign(p->weights, p->weights + p->weights_count);
    if (p->mol_offsets)
        c->mol_offsets.assign(p->mol_offsets, p->mol_offsets + c->nmol + 1);
    else
        c->mol_offsets = {0, c->n};
    c->mol_of.assign(c->n, 0);
    for (int m = 0; m < c->nmol; ++m)
        for (int i = c->mol_offsets[m]; i < c->mol_offsets[m + 1]; ++i) c->mol_of[i] = m;

    hipError_t e = hipSuccess;
    if (p->stream || p->use_stream) {
        c->stream = (hipStream_t)p->stream;
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            nnp_status r = hip_fail(c, e, "hipStreamCreate");
            fprintf(stderr, "nnp_create: %s\n", c->err.c_str());
            delete c;
            return r;
        }
        c->own_stream = true;
    }
    const size_t n = c->n, cap = c->cap, nm = c->nmol;
    Sys& S = c->S;
    S.n = c->n;
    S.nmol = c->nmol;
    S.cap = c->cap;
    S.rebuild_every = c->rebuild_every;
    S.rlist2 = (float)((5.2 + c->skin) * (5.2 + c->skin));
    S.half_skin2 = (float)(0.25 * c->skin * c->skin);
#define ALLOC(field, type, count)                                         \
    S.field = (type)dev_alloc(c, sizeof(*S.field) * (size_t)(count), &e); \
    if (e != hipSuccess) goto oom;
    ALLOC(pos, double4*, n)
    ALLOC(vel, double4*, n)
    ALLOC(frc, double4*, n)
    ALLOC(ref, float4*, n)
    ALLOC(kinv, const double*, n)
    ALLOC(mass, const double*, n)
    ALLOC(mol, const int*, n)
    ALLOC(mrange, const int2*, nm * 4)
    ALLOC(tiles, const int4*, n)
    ALLOC(tile_atoms, const int*, (size_t)n * kTileCap)
    ALLOC(tile_mol, const int*, n)
    ALLOC(work, int*, n)
    ALLOC(nbr, int*, n * cap)
    ALLOC(ncnt, int*, n)
    ALLOC(facc, unsigned long long*, (size_t)kFaccCopies * 4 * n)
    ALLOC(Ei, float*, n)
    ALLOC(Uring, double*, (size_t)kRing * nm)
    ALLOC(Kring, double*, (size_t)kRing * nm)
    ALLOC(Eacc, double*, 2 * nm)
    ALLOC(Kacc, double*, 2 * nm)
    ALLOC(Ecur, double*, nm)
    ALLOC(Kcur, double*, nm)
    ALLOC(perm, const int*, n)
    ALLOC(stage, double*, 3 * n)
    ALLOC(molgrid, const int*, nm)
    ALLOC(st, StepState*, 1)
    ALLOC(w32, const float*, (size_t)4 * W32Layout::Stride)
    S.wfrag = dev_alloc(c, (size_t)4 * 2 * FragLayout::Count * 1024, &e);
    if (e != hipSuccess) goto oom;
    S.wfrag8 = dev_alloc(c, (size_t)4 * FragLayout::Count * 512, &e);
    if (e != hipSuccess) goto oom;
    ALLOC(wscale8, const float*, 4 * 6)
    if (c->path == NNP_PATH_PLAIN) {
        ALLOC(G, float*, n * kNumFeat)
        ALLOC(dG, float*, n * kNumFeat)
    }
    if (c->path == NNP_PATH_SPLIT && split_buffers(c) != NNP_OK) {
        e = hipErrorOutOfMemory;
        goto oom;
    }
#undef ALLOC
    {
        std::vector<float> w32, ws8;
        std::vector<uint16_t> frag;
        std::vector<uint8_t> frag8;
        build_weights(c->weights, w32, frag, frag8, ws8);
        e = hipMemcpy((void*)S.w32, w32.data(), sizeof(float) * w32.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((void*)S.wfrag, frag.data(), sizeof(uint16_t) * frag.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((void*)S.wfrag8, frag8.data(), frag8.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((void*)S.wscale8, ws8.data(), sizeof(float) * ws8.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) goto oom;
    }
    *out = c;
    return NNP_OK;
oom:
    {
        nnp_status r = hip_fail(c, e, "device allocation");
        fprintf(stderr, "nnp_create: %s\n", c->err.c_str());
        nnp_destroy(c);
        return r;
    }
}

void nnp_destroy(nnp_context* c)
{
    if (!c) return;
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static[c->static_dev].owner == c) g_static[c->static_dev].owner = nullptr;
    }
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_rebalance_buffers(c);
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    for (auto& b : c->bufs) (void)hipFree(b.p);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

nnp_status nnp_energy_device(nnp_context* c, const void* d_pos, int is_f64, double* d_energy, int keep)
{
    if (!c) return NNP_ERR_ARG;
    if (!d_pos || !d_energy) return fail(c, NNP_ERR_ARG, "d_pos and d_energy are required");
    if (!c->laid_out) return fail(c, NNP_ERR_STATE, "set positions once with nnp_set_state or nnp_compute first");
    if (keep && (!c->S.G || !c->S.dG)) {
        hipError_t e = hipSuccess;
        c->S.G = (float*)dev_alloc(c, sizeof(float) * (size_t)c->n * kNumFeat, &e);
        if (e == hipSuccess) c->S.dG = (float*)dev_alloc(c, sizeof(float) * (size_t)c->n * kNumFeat, &e);
        if (e != hipSuccess) return hip_fail(c, e, "stored-mode buffers");
    }
    HIP_TRY(c, launch_positions_in(c->S, d_pos, is_f64 ? 1 : 0, c->stream));
    HIP_TRY(c, launch_invalidate_lists(c->S, c->stream));
    if (keep) {
        // plain-path kernels keep G and dE/dG; the pair list stays marked for
        // rebuild so the adjoint's gather records the reverse slots
        HIP_TRY(c, launch_store_forward(c->S, mode_of(c), c->T, c->stream));
        HIP_TRY(c, launch_gather_integrate(c->S, 0.0, 0, c->stream, false));
    } else {
        HIP_TRY(c, enqueue_eval(c, false));
        HIP_TRY(c, launch_gather_integrate(c->S, 0.0, 0, c->stream, false));
    }
    HIP_TRY(c, launch_energy_out(c->S, d_energy, c->stream));
    c->diff_state = keep ? 2 : 1;
    c->forces_current = false;
    c->kick_pending = false;
    return NNP_OK;
}

nnp_status nnp_energy_device_static(nnp_context* c, const void* d_pos, int is_f64, double* d_energy)
{
    if (!c) return NNP_ERR_ARG;
    if (!d_pos || !d_energy) return fail(c, NNP_ERR_ARG, "d_pos and d_energy are required");
    if (!c->laid_out) return fail(c, NNP_ERR_STATE, "set positions once with nnp_set_state or nnp_compute first");
    if (c->n > kStaticAtoms)
        return fail(c, NNP_ERR_ARG, "nnp_energy_device_static holds at most " + std::to_string(kStaticAtoms) +
                                        " atoms (context has " + std::to_string(c->n) + ")");
    int dev = 0;
    HIP_TRY(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticDevices) return fail(c, NNP_ERR_UNSUPPORTED, "device ordinal beyond the scratch table");
    float* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        StaticScratch& x = g_static[dev];
        if (!x.ptr) {
            // once per device, with that device current: the array's address
            // on this GPU
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) return hip_fail(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
            x.ptr = static_cast<float*>(p);
        }
        x.owner = c;
        x.gen += 1;
        c->static_dev = dev;
        c->static_gen = x.gen;
        base = x.ptr;
    }
    // the kernels write every element of G and dE/dG they later read:
    // nothing in the scratch has to start at zero
    Sys S = c->S;
    S.G = base;
    S.dG = base + (size_t)c->n * kNumFeat;
    HIP_TRY(c, launch_positions_in(S, d_pos, is_f64 ? 1 : 0, c->stream));
    HIP_TRY(c, launch_invalidate_lists(S, c->stream));
    HIP_TRY(c, launch_store_forward(S, mode_of(c), c->T, c->stream));
    HIP_TRY(c, launch_gather_integrate(S, 0.0, 0, c->stream, false));
    HIP_TRY(c, launch_energy_out(S, d_energy, c->stream));
    c->diff_state = 3;
    c->forces_current = false;
    c->kick_pending = false;
    return NNP_OK;
}

nnp_status nnp_forces_device(nnp_context* c, double* d_forces)
{
    if (!c) return NNP_ERR_ARG;
    if (!d_forces) return fail(c, NNP_ERR_ARG, "d_forces is required");
    if (c->diff_state == 0) return fail(c, NNP_ERR_STATE, "call nnp_energy_device first");
    if (c->diff_state == 3) {
        // allocation-free stored mode: dE/dG sits in the device's static
        // scratch, unless a later call has reused it
        Sys S = c->S;
        {
            std::lock_guard<std::mutex> lk(g_static_mu);
            const StaticScratch& x = g_static[c->static_dev];
            if (x.owner != c || x.gen != c->static_gen)
                return fail(c, NNP_ERR_STATE, "the static scratch was reused by a later nnp_energy_device_static call");
            S.G = x.ptr;
            S.dG = x.ptr + (size_t)c->n * kNumFeat;
        }
        HIP_TRY(c, launch_adjoint(S, c->stream));
    } else if (c->diff_state == 2) {
        // stored mode: the pair list and reverse slots of the forward are
        // current; the adjoint reads the kept dE/dG
        HIP_TRY(c, launch_adjoint(c->S, c->stream));
    } else {
        HIP_TRY(c, launch_invalidate_lists(c->S, c->stream));
        HIP_TRY(c, enqueue_eval(c, true));
    }
    HIP_TRY(c, launch_gather_integrate(c->S, 0.0, 0, c->stream, true));
    HIP_TRY(c, launch_forces_out(c->S, d_forces, c->stream));
    c->forces_current = true;
    return NNP_OK;
}

nnp_status nnp_set_state(nnp_context* c, const double* pos, const double* vel)
{
    if (!c) return NNP_ERR_ARG;
    c->diff_state = 0;
    if (vel)
        for (int i = 0; i < 3 * c->n; ++i)
            if (!std::isfinite(vel[i])) return fail(c, NNP_ERR_NONFINITE, "non-finite velocity component");
    if (pos) {
        nnp_status s = upload_positions(c, pos);
        if (s != NNP_OK) return s;
        hipError_t e = launch_invalidate_lists(c->S, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "invalidate");
        c->forces_current = false;
        c->kick_pending = false;
        // a new trajectory starts from the initial tiling with no recorded work
        if (balanced_tiles(c)) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            const nnp_status ts = upload_tiles(c, std::vector<int4>(c->tiles_init));
            if (ts != NNP_OK) return ts;
            HIP_TRY(c, hipMemset(c->S.work, 0, sizeof(int) * c->n));
        }
    }
    if (vel) {
        if (!c->laid_out) return fail(c, NNP_ERR_STATE, "set positions before velocities");
        std::vector<double4> v4(c->n);
        for (int k = 0; k < c->n; ++k) {
            const int i = c->perm[k];
            v4[k] = make_double4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.0);
        }
        HIP_TRY(c, hipMemcpyAsync(c->S.vel, v4.data(), sizeof(double4) * c->n, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (c->kick_pending) c->forces_current = true;  // forces unchanged, velocities replaced
    }
    c->err.clear();
    return NNP_OK;
}

nnp_status nnp_set_box(nnp_context* c, const double* box)
{
    if (!c) return NNP_ERR_ARG;
    const double rl = 5.2 + c->skin;
    if (box) {
        if (c->nmol != 1) return fail(c, NNP_ERR_UNSUPPORTED, "a periodic box needs n_molecules == 1");
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(box[d]) || !(box[d] >= 2.0 * rl)) {
                char b[160];
                snprintf(b, sizeof b, "box edges must be finite and >= 2 (5.2 + skin) = %.2f A", 2.0 * rl);
                return fail(c, NNP_ERR_ARG, b);
            }
    }
    const bool same = box ? (c->S.periodic && box[0] == c->box[0] && box[1] == c->box[1] && box[2] == c->box[2])
                          : !c->S.periodic;
    if (same) return NNP_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<double> pos;
    if (c->laid_out && !box) {
        // back to the gas phase: grids follow the current positions
        std::vector<double4> p4(c->n);
        HIP_TRY(c, hipMemcpy(p4.data(), c->S.pos, sizeof(double4) * c->n, hipMemcpyDeviceToHost));
        pos.resize(3 * (size_t)c->n);
        for (int k = 0; k < c->n; ++k) {
            const int i = c->perm[k];
            pos[3 * i] = p4[k].x;
            pos[3 * i + 1] = p4[k].y;
            pos[3 * i + 2] = p4[k].z;
        }
    }
    c->S.periodic = box ? 1 : 0;
    for (int d = 0; d < 3; ++d) c->box[d] = box ? box[d] : 0.0;
    c->S.box = make_double3(c->box[0], c->box[1], c->box[2]);
    c->S.ibox = box ? make_double3(1.0 / box[0], 1.0 / box[1], 1.0 / box[2]) : make_double3(0.0, 0.0, 0.0);
    if (c->laid_out) {
        const nnp_status gs = setup_grids(c, pos.empty() ? nullptr : pos.data());
        if (gs != NNP_OK) return gs;
        HIP_TRY(c, launch_invalidate_lists(c->S, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        c->forces_current = false;
        c->kick_pending = false;
    }
    // captured graphs hold the old box in their kernel arguments
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
    c->err.clear();
    return NNP_OK;
}

nnp_status nnp_compute(nnp_context* c, const double* pos, const double* box, double* energy, double* forces)
{
    if (!c) return NNP_ERR_ARG;
    c->diff_state = 0;
    if (box) {
        const nnp_status bs = nnp_set_box(c, box);
        if (bs != NNP_OK) return bs;
    }
    if (!pos || !energy) return fail(c, NNP_ERR_ARG, "pos and energy are required");
    if (forces && c->energy_only) return fail(c, NNP_ERR_ARG, "the context returns energy only: forces must be NULL");
    nnp_status s = upload_positions(c, pos);
    if (s != NNP_OK) return s;
    HIP_TRY(c, launch_invalidate_lists(c->S, c->stream));
    const bool grad = !c->energy_only;
    s = full_compute(c, grad);
    if (s != NNP_OK) return s;
    std::vector<double4> f4;
    if (forces) {
        f4.resize(c->n);
        HIP_TRY(c, hipMemcpyAsync(f4.data(), c->S.frc, sizeof(double4) * c->n, hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, launch_energy_flush(c->S, c->stream));
    HIP_TRY(c, hipMemcpyAsync(energy, c->S.Ecur, sizeof(double) * c->nmol, hipMemcpyDeviceToHost, c->stream));
    s = check_device_flags(c);
    if (s != NNP_OK) return s;
    if (forces)
        for (int k = 0; k < c->n; ++k) {
            const int i = c->perm[k];
            forces[3 * i] = f4[k].x;
            forces[3 * i + 1] = f4[k].y;
            forces[3 * i + 2] = f4[k].z;
        }
    c->forces_current = grad;
    c->kick_pending = false;
    c->err.clear();
    return NNP_OK;
}

nnp_status nnp_compute_device(nnp_context* c, const void* d_pos, int is_f64, double* d_energy, double* d_forces)
{
    if (!c) return NNP_ERR_ARG;
    c->diff_state = 0;
    if (!d_pos || !d_energy) return fail(c, NNP_ERR_ARG, "d_pos and d_energy are required");
    if (!c->laid_out) return fail(c, NNP_ERR_STATE, "set positions once with nnp_set_state or nnp_compute first");
    if (d_forces && c->energy_only)
        return fail(c, NNP_ERR_ARG, "the context returns energy only: d_forces must be NULL");
    HIP_TRY(c, launch_positions_in(c->S, d_pos, is_f64 ? 1 : 0, c->stream));
    HIP_TRY(c, launch_invalidate_lists(c->S, c->stream));
    const bool grad = d_forces != nullptr;
    const nnp_status fs = full_compute(c, grad);
    if (fs != NNP_OK) return fs;
    if (grad) HIP_TRY(c, launch_forces_out(c->S, d_forces, c->stream));
    HIP_TRY(c, launch_energy_out(c->S, d_energy, c->stream));
    c->forces_current = grad;
    c->kick_pending = false;
    return NNP_OK;
}

nnp_status nnp_step(nnp_context* c, double dt, int32_t nsteps, int32_t use_graph)
{
    if (!c) return NNP_ERR_ARG;
    c->diff_state = 0;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, NNP_ERR_ARG, "dt must be finite and > 0");
    if (nsteps < 0) return fail(c, NNP_ERR_ARG, "n_steps must be >= 0");
    if (!c->laid_out) return fail(c, NNP_ERR_STATE, "set positions before stepping");
    if (nsteps == 0) return NNP_OK;
    if (!c->forces_current) {
        const nnp_status fs = full_compute(c);
        if (fs != NNP_OK) return fs;
        c->forces_current = true;
    }
    const int B = std::min<int>(nsteps, kGraphBlock);
    if (!c->extra.empty()) {
        for (int left = nsteps; left > 0; left -= B) {
            nnp_status bs = rebalance_tiles(c);
            if (bs == NNP_OK) bs = steps_with_extra(c, dt, std::min(left, B));
            if (bs != NNP_OK) return bs;
        }
        c->kick_pending = true;
        return NNP_OK;
    }
    if (!use_graph || c->stream == nullptr) {
        // blocks of at most kGraphBlock steps, as with graphs (tile balancing between
        // blocks gives graph and eager runs the same trajectory)
        for (int left = nsteps; left > 0; left -= B) {
            const nnp_status bs = rebalance_tiles(c);
            if (bs != NNP_OK) return bs;
            HIP_TRY(c, enqueue_steps(c, dt, std::min(left, B), true));
        }
        c->kick_pending = true;
        return NNP_OK;
    }
    auto run_block = [&](int len) -> nnp_status {
        hipGraphExec_t x = nullptr;
        const nnp_status gs = block_graph(c, dt, len, &x);
        if (gs != NNP_OK) return gs;
        HIP_TRY(c, hipGraphLaunch(x, c->stream));
        return NNP_OK;
    };
    int left = nsteps;
    while (left > 0) {
        const int len = left >= B ? B : left;
        nnp_status s = rebalance_tiles(c);
        if (s != NNP_OK) return s;
        s = run_block(len);
        if (s != NNP_OK) return s;
        left -= len;
    }
    c->kick_pending = true;
    return NNP_OK;
}

nnp_status nnp_capture(nnp_context* c, double dt, int32_t nsteps)
{
    if (!c) return NNP_ERR_ARG;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, NNP_ERR_ARG, "dt must be finite and > 0");
    if (nsteps < 0) return fail(c, NNP_ERR_ARG, "n_steps must be >= 0");
    if (c->stream == nullptr) return fail(c, NNP_ERR_STATE, "graphs cannot be captured on the null stream");
    if (!c->extra.empty()) return fail(c, NNP_ERR_STATE, "steps with extra force providers are not captured");
    if (nsteps == 0) return NNP_OK;
    const int B = std::min<int>(nsteps, kGraphBlock);
    hipGraphExec_t x = nullptr;
    nnp_status s = block_graph(c, dt, B, &x);
    if (s == NNP_OK && nsteps % B != 0) s = block_graph(c, dt, nsteps % B, &x);
    if (s == NNP_OK) c->err.clear();
    return s;
}

nnp_status nnp_add_force(nnp_context* c, nnp_force_fn fn, void* user, double* d_pos, double* d_forces,
                          double* d_energy)
{
    if (!c) return NNP_ERR_ARG;
    if (!fn || !d_pos || !d_forces || !d_energy) return fail(c, NNP_ERR_ARG, "fn and the three buffers are required");
    if (c->extra.size() >= 8) return fail(c, NNP_ERR_ARG, "at most 8 extra force providers");
    c->extra.push_back({fn, user, d_pos, d_forces, d_energy});
    c->forces_current = false;
    c->err.clear();
    return NNP_OK;
}

nnp_status nnp_clear_forces(nnp_context* c)
{
    if (!c) return NNP_ERR_ARG;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!c->extra.empty()) c->forces_current = false;
    c->extra.clear();
    return NNP_OK;
}

nnp_status nnp_set_thermostat(nnp_context* c, double temperature, double friction, uint64_t seed)
{
    if (!c) return NNP_ERR_ARG;
    if (!(temperature >= 0.0) || !std::isfinite(temperature))
        return fail(c, NNP_ERR_ARG, "temperature must be finite and >= 0");
    if (!(friction >= 0.0) || !std::isfinite(friction)) return fail(c, NNP_ERR_ARG, "friction must be finite and >= 0");
    c->S.gamma = friction * 1e-3;           // 1/ps -> 1/fs
    c->S.kT = 8.617333262e-5 * temperature;  // Boltzmann constant in eV/K
    c->S.seed = seed;
    c->err.clear();
    return NNP_OK;
}

nnp_status nnp_get_state(nnp_context* c, double* pos, double* vel, double* forces, double* pot, double* kin)
{
    if (!c) return NNP_ERR_ARG;
    if (!c->laid_out) return fail(c, NNP_ERR_STATE, "no positions set");
    std::vector<double4> p4, v4, f4;
    if (pos) {
        p4.resize(c->n);
        HIP_TRY(c, hipMemcpyAsync(p4.data(), c->S.pos, sizeof(double4) * c->n, hipMemcpyDeviceToHost, c->stream));
    }
    if (vel) {
        v4.resize(c->n);
        HIP_TRY(c, hipMemcpyAsync(v4.data(), c->S.vel, sizeof(double4) * c->n, hipMemcpyDeviceToHost, c->stream));
    }
    if (forces) {
        f4.resize(c->n);
        HIP_TRY(c, hipMemcpyAsync(f4.data(), c->S.frc, sizeof(double4) * c->n, hipMemcpyDeviceToHost, c->stream));
    }
    if (pot || kin) HIP_TRY(c, launch_energy_flush(c->S, c->stream));
    if (pot) HIP_TRY(c, hipMemcpyAsync(pot, c->S.Ecur, sizeof(double) * c->nmol, hipMemcpyDeviceToHost, c->stream));
    if (kin) HIP_TRY(c, hipMemcpyAsync(kin, c->S.Kcur, sizeof(double) * c->nmol, hipMemcpyDeviceToHost, c->stream));
    nnp_status s = check_device_flags(c);
    if (s != NNP_OK) return s;
    for (int k = 0; k < c->n; ++k) {
        const int i = c->perm[k];
        if (pos) {
            pos[3 * i] = p4[k].x;
            pos[3 * i + 1] = p4[k].y;
            pos[3 * i + 2] = p4[k].z;
        }
        if (vel) {
            vel[3 * i] = v4[k].x;
            vel[3 * i + 1] = v4[k].y;
            vel[3 * i + 2] = v4[k].z;
        }
        if (forces) {
            forces[3 * i] = f4[k].x;
            forces[3 * i + 1] = f4[k].y;
            forces[3 * i + 2] = f4[k].z;
        }
    }
    return NNP_OK;
}

nnp_status nnp_energy_log(nnp_context* c, int32_t count, double* U, double* K, int32_t* written)
{
    if (!c || !U || !K || !written || count < 0) return fail(c, NNP_ERR_ARG, "bad arguments");
    *written = 0;
    HIP_TRY(c, launch_energy_flush(c->S, c->stream));
    // energies of steps whose environments were clamped (or not finite) are
    // not handed out: the sticky device flags are reported here too
    const nnp_status f = check_device_flags(c);
    if (f != NNP_OK) return f;
    StepState st;
    HIP_TRY(c, hipMemcpyAsync(&st, c->S.st, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // the most recent evaluation sits in last_slot; evaluations of steps are
    // consecutive slots
    const int have = st.n_eval > 0 ? std::min(st.last_slot + 1, kRing) : 0;
    const int w = std::min(count, have);
    const size_t nm = c->nmol;
    std::vector<double> u(nm), k(nm);
    for (int q = 0; q < w; ++q) {
        const int slot = ((st.last_slot - (w - 1 - q)) % kRing + kRing) % kRing;
        HIP_TRY(c, hipMemcpy(U + (size_t)q * nm, c->S.Uring + (size_t)slot * nm, sizeof(double) * nm, hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(K + (size_t)q * nm, c->S.Kring + (size_t)slot * nm, sizeof(double) * nm, hipMemcpyDeviceToHost));
    }
    *written = w;
    return NNP_OK;
}

nnp_status nnp_stats(nnp_context* c, int64_t* stats)
{
    if (!c || !stats) return fail(c, NNP_ERR_ARG, "bad arguments");
    StepState st;
    HIP_TRY(c, hipMemcpyAsync(&st, c->S.st, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    stats[0] = st.n_eval;
    stats[1] = st.n_rebuild;
    stats[2] = st.n_forced;
    stats[3] = st.step;
    stats[4] = st.max_ns;
    stats[5] = st.max_nr;
    stats[6] = st.max_na;
    return NNP_OK;
}

nnp_status nnp_get_config(const nnp_context* c, int32_t* config)
{
    if (!c || !config) return NNP_ERR_ARG;
    config[0] = (int32_t)c->path;
    config[1] = c->T;
    config[2] = 16 * c->nblk;
    return NNP_OK;
}

nnp_status nnp_debug_descriptors(nnp_context* c, const double* pos, float* G)
{
    if (!c || !pos || !G) return fail(c, NNP_ERR_ARG, "bad arguments");
    nnp_status s = upload_positions(c, pos);
    if (s != NNP_OK) return s;
    Sys S = c->S;
    float* dG = nullptr;
    if (!S.G) {
        HIP_TRY(c, hipMalloc(&dG, sizeof(float) * (size_t)c->n * kNumFeat));
        S.G = dG;
    }
    hipError_t e = launch_invalidate_lists(S, c->stream);
    if (e == hipSuccess) e = launch_descriptors_only(S, c->stream);
    std::vector<float> tmp((size_t)c->n * kNumFeat);
    if (e == hipSuccess)
        e = hipMemcpyAsync(tmp.data(), S.G, sizeof(float) * tmp.size(), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (dG) (void)hipFree(dG);
    if (e != hipSuccess) return hip_fail(c, e, "descriptors");
    s = check_device_flags(c);
    if (s != NNP_OK) return s;
    for (int k = 0; k < c->n; ++k)
        std::memcpy(G + (size_t)c->perm[k] * kNumFeat, tmp.data() + (size_t)k * kNumFeat, sizeof(float) * kNumFeat);
    // the lists were built outside a step; the next evaluation rebuilds them
    HIP_TRY(c, launch_invalidate_lists(c->S, c->stream));
    c->forces_current = false;
    c->kick_pending = false;
    return NNP_OK;
}

nnp_status nnp_debug_atom_energies(nnp_context* c, double* Ei)
{
    if (!c || !Ei) return fail(c, NNP_ERR_ARG, "bad arguments");
    std::vector<float> e(c->n);
    HIP_TRY(c, hipMemcpyAsync(e.data(), c->S.Ei, sizeof(float) * c->n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < c->n; ++k) Ei[c->perm[k]] = e[k];
    return NNP_OK;
}

nnp_status nnp_device_bytes(nnp_context* c, int64_t* bytes)
{
    if (!c || !bytes) return fail(c, NNP_ERR_ARG, "bad arguments");
    int64_t b = 0;
    for (auto& x : c->bufs) b += (int64_t)x.bytes;
    *bytes = b;
    return NNP_OK;
}

nnp_status nnp_debug_fp8_encode(const float* x, int32_t n, uint8_t* device_out, uint8_t* host_out)
{
    if (!x || n <= 0 || (!device_out && !host_out)) return NNP_ERR_ARG;
    if (host_out)
        for (int i = 0; i < n; ++i) host_out[i] = e4m3_encode(x[i]);
    if (!device_out) return NNP_OK;
    float* dx = nullptr;
    uint8_t* dq = nullptr;
    if (hipMalloc(&dx, sizeof(float) * n) != hipSuccess) return NNP_ERR_OOM;
    if (hipMalloc(&dq, n) != hipSuccess) {
        (void)hipFree(dx);
        return NNP_ERR_OOM;
    }
    hipError_t e = hipMemcpy(dx, x, sizeof(float) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_fp8_encode(dx, n, dq, nullptr);
    if (e == hipSuccess) e = hipMemcpy(device_out, dq, n, hipMemcpyDeviceToHost);
    (void)hipFree(dx);
    (void)hipFree(dq);
    return e == hipSuccess ? NNP_OK : NNP_ERR_HIP;
}

nnp_status nnp_time_kernels(nnp_context* c, int32_t reps, double* ms)
{
    if (!c || !ms || reps < 1) return fail(c, NNP_ERR_ARG, "bad arguments");
    if (!c->laid_out) return fail(c, NNP_ERR_STATE, "set positions first");
    HIP_TRY(c, enqueue_compute(c, true));
    hipEvent_t e0, e1, e2;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    HIP_TRY(c, hipEventCreate(&e2));
    HIP_TRY(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps; ++r) HIP_TRY(c, enqueue_eval(c, true));
    HIP_TRY(c, hipEventRecord(e1, c->stream));
    for (int r = 0; r < reps; ++r) HIP_TRY(c, launch_gather_integrate(c->S, 0.0, 0, c->stream));
    HIP_TRY(c, hipEventRecord(e2, c->stream));
    HIP_TRY(c, hipEventSynchronize(e2));
    float a = 0.f, b = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&a, e0, e1));
    HIP_TRY(c, hipEventElapsedTime(&b, e1, e2));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    ms[0] = a / reps;
    ms[1] = b / reps;
    // the timed evaluations summed their forces without a gather in between:
    // one complete evaluation leaves the forces and energies consistent
    HIP_TRY(c, enqueue_compute(c, true));
    c->forces_current = c->extra.empty();
    c->kick_pending = false;
    return check_device_flags(c);
}

nnp_status nnp_time_steps(nnp_context* c, double dt, int32_t nsteps, double* ms)
{
    if (!c || !ms || nsteps < 1) return fail(c, NNP_ERR_ARG, "bad arguments");
    if (!c->extra.empty()) return fail(c, NNP_ERR_UNSUPPORTED, "timed steps cover the network only (extra forces set)");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, NNP_ERR_ARG, "dt must be finite and > 0");
    if (!c->laid_out) return fail(c, NNP_ERR_STATE, "set positions before stepping");
    c->diff_state = 0;
    if (!c->forces_current) {
        HIP_TRY(c, enqueue_compute(c, true));
        c->forces_current = true;
    }
    {
        const nnp_status bs = rebalance_tiles(c);  // as at the start of a block of nnp_step
        if (bs != NNP_OK) return bs;
    }
    // per step: start / end of the evaluation kernel(s) and of the gather /
    // integration kernel, stamped by the dispatches themselves
    std::vector<hipEvent_t> ev(4 * (size_t)nsteps, nullptr);
    hipError_t e = hipSuccess;
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    if (e == hipSuccess) e = launch_kickdrift(c->S, dt, c->stream);
    for (int i = 0; i < nsteps && e == hipSuccess; ++i) {
        e = launch_eval(c->S, (int)c->path, mode_of(c), c->T, true, c->stream, ev[4 * i],
                        ev[4 * i + 1]);
        if (e == hipSuccess)
            e = launch_gather_integrate(c->S, dt, i == nsteps - 1 ? 1 : 2, c->stream, true, ev[4 * i + 2],
                                        ev[4 * i + 3]);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[4 * (size_t)nsteps - 1]);
    double sum_eval = 0.0, sum_gather = 0.0;
    for (int i = 0; i < nsteps && e == hipSuccess; ++i) {
        float a = 0.f, b = 0.f;
        e = hipEventElapsedTime(&a, ev[4 * i], ev[4 * i + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[4 * i + 2], ev[4 * i + 3]);
        sum_eval += a;
        sum_gather += b;
    }
    float total = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&total, ev[0], ev[4 * (size_t)nsteps - 1]);
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(c, e, "timed steps");
    ms[0] = sum_eval / nsteps;
    ms[1] = sum_gather / nsteps;
    ms[2] = (double)total / nsteps;
    c->kick_pending = true;
    return check_device_flags(c);
}

nnp_status nnp_autotune(nnp_context* c, const char* cache_path, int32_t* choice)
{
    if (!c) return NNP_ERR_ARG;
    if (!c->laid_out) return fail(c, NNP_ERR_STATE, "set positions before autotuning");
    // systems whose atom and molecule counts fall in the same power-of-two
    // buckets share a tuned configuration; fused and split tune together
    auto bucket = [](int v) {
        int b = 0;
        while ((2 << b) <= v) ++b;
        return b;
    };
    const bool bf = split_dtype_ok(c->dtype);
    const int family = c->path == NNP_PATH_PLAIN ? 0 : 1;
    const std::string key = "nb" + std::to_string(bucket(c->n)) + "_mb" + std::to_string(bucket(c->nmol)) + "_f" +
                            std::to_string(family) + "_d" + std::to_string((int)c->dtype) + "_pbc" +
                            std::to_string(c->S.periodic ? 1 : 0);
    struct Cand {
        nnp_path path;
        int T, nblk;
    };
    auto valid = [&](const Cand& k) {
        if (family == 0) return k.path == NNP_PATH_PLAIN && (k.T == 8 || k.T == 16);
        if (k.path == NNP_PATH_FUSED) return fused_tile_ok(k.T, c->dtype);
        return k.path == NNP_PATH_SPLIT && bf && split_tile_ok(k.T) && k.nblk >= 1 && k.nblk <= 4;
    };
    auto apply = [&](const Cand& k, bool cached) {
        nnp_status s = retile(c, k.T, k.path, k.nblk);
        if (s != NNP_OK) return s;
        if (choice) {
            choice[0] = (int32_t)k.path;
            choice[1] = k.T;
            choice[2] = 16 * k.nblk;
            choice[3] = cached ? 1 : 0;
        }
        return NNP_OK;
    };
    auto field = [](const std::string& line, const char* name, int* out) {
        const std::string pat = std::string("\"") + name + "\": ";
        const size_t p = line.find(pat);
        if (p == std::string::npos) return false;
        *out = std::atoi(line.c_str() + p + pat.size());
        return true;
    };
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            if (line.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
            int pa = 0, T = 0, nt = 0;
            if (!field(line, "path", &pa) || !field(line, "atoms_per_tile", &T) || !field(line, "network_tile", &nt))
                continue;
            const Cand k{(nnp_path)pa, T, nt / 16};
            if (valid(k)) return apply(k, true);
        }
    }
    std::vector<Cand> cand;
    if (family == 0) {
        cand = {{NNP_PATH_PLAIN, 8, c->nblk}, {NNP_PATH_PLAIN, 16, c->nblk}};
    } else {
        for (int T : {4, 5, 8, 10, 12, 13, 14, 15, 16})
            if (fused_tile_ok(T, c->dtype)) cand.push_back({NNP_PATH_FUSED, T, c->nblk});
        if (bf)
            for (int T : {4, 5, 7, 10})
                for (int nb : {2, 4}) cand.push_back({NNP_PATH_SPLIT, T, nb});
    }
    double best = 1e300;
    Cand bestk = {c->path, c->T, c->nblk};
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    std::ostringstream times;
    for (const Cand& k : cand) {
        nnp_status s = retile(c, k.T, k.path, k.nblk);
        if (s != NNP_OK) return s;
        HIP_TRY(c, enqueue_eval(c, true));  // warm-up (also builds the lists)
        HIP_TRY(c, launch_gather_integrate(c->S, 0.0, 0, c->stream));
        HIP_TRY(c, hipEventRecord(e0, c->stream));
        const int reps = 20;
        for (int r = 0; r < reps; ++r) {
            HIP_TRY(c, enqueue_eval(c, true));
            HIP_TRY(c, launch_gather_integrate(c->S, 0.0, 0, c->stream));
        }
        HIP_TRY(c, hipEventRecord(e1, c->stream));
        HIP_TRY(c, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
        times << (times.tellp() > 0 ? ", " : "") << "\""
              << (k.path == NNP_PATH_SPLIT ? "split" : k.path == NNP_PATH_FUSED ? "fused" : "plain") << "/" << k.T;
        if (k.path == NNP_PATH_SPLIT) times << "x" << 16 * k.nblk;
        times << "\": " << ms / reps;
        if (ms < best) {
            best = ms;
            bestk = k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    nnp_status s = apply(bestk, false);
    if (s != NNP_OK) return s;
    if (!c->extra.empty()) c->forces_current = false;  // the timed evaluations had no extra forces
    nnp_status f = check_device_flags(c);
    if (f != NNP_OK) return f;
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << "{\"key\": \"" << key << "\", \"path\": " << (int)bestk.path << ", \"atoms_per_tile\": " << bestk.T
          << ", \"network_tile\": " << 16 * bestk.nblk << ", \"ms_per_eval\": {" << times.str() << "}}\n";
    }
    return NNP_OK;
}

}  // extern "C"
