// nnp_device.h -- wave-level device functions of one energy/force evaluation.
//
// One wavefront (64 lanes) owns one centre atom for the pair-list build, the
// environment load, the descriptors and the adjoint.  The network stage is a
// workgroup-wide operation over a tile of atoms of one element.
//
// Model (the symmetry-function network potential behind the paper's
// force-provider contract, Methods section):
//   radial   G[16 s_j + k]       = sum_j exp(-16 (r_ij - R_k)^2) fc(r_ij; 5.2),  R_k = 0.9 + 0.28 k
//   angular  G[64 + 32 p + 8m + n] = sum_{j<k} 2^-31 (1 + c' cos t_n + sqrt(1-c'^2) sin t_n)^32
//                                  * exp(-8 ((r_ij + r_ik)/2 - Q_m)^2) fc(r_ij; 3.5) fc(r_ik; 3.5),
//            c' = 0.95 cos(theta_jik), t_n = (2n+1) pi/16, Q_m = 0.9 + 0.65 m
//   network  384 -> 160 -> 128 -> 96 -> 1, CELU(0.1); E = sum_i E_i; F = -dE/dx.
#pragma once

#include <type_traits>

#include "nnp_internal.h"

namespace nnp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

__constant__ static const float kSecCos[8] = {9.807852507e-01f, 8.314695954e-01f, 5.555702448e-01f,
                                               1.950903237e-01f, -1.950903237e-01f, -5.555702448e-01f,
                                               -8.314695954e-01f, -9.807852507e-01f};
__constant__ static const float kSecSin[8] = {1.950903237e-01f, 5.555702448e-01f, 8.314695954e-01f,
                                               9.807852507e-01f, 9.807852507e-01f, 8.314695954e-01f,
                                               5.555702448e-01f, 1.950903237e-01f};
constexpr float kTwoPowM31 = 4.656612873e-10f;  // 2^(1 - zeta), zeta = 32
constexpr float kPi = 3.14159265358979f;

// Environment of one centre atom, in LDS.  Entries are the neighbours within
// 5.2 A in ascending internal index (hence grouped by element).
struct Env {
    float4 geo[kRadMax];            // unit vector to the neighbour, distance
    float2 fcr[kRadMax];            // fc(r; 5.2), dfc/dr
    float2 afc[kAngMax];            // fc(r; 3.5), dfc/dr of angular entries
    int nid[kRadMax];               // internal index of the neighbour
    unsigned short info[kRadMax];   // element | (slot in the pair list) << 2
    unsigned char ang[kAngMax];     // radial-entry index of neighbours within 3.5 A
    int nR, nA, nS;                 // radial entries, angular entries, pair-list length
    int aseg[5];                    // angular entries of element s: [aseg[s], aseg[s+1])
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Orders LDS accesses of the lanes of one wavefront: without it the compiler
// may move a lane's read of a value another lane wrote above that write.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0));
}

// Adds neighbour candidate to the wave's environment (called for every
// accepted pair-list slot, in slot order, by all 64 lanes together).  The
// relative vector is formed in FP64 from the master positions and rounded to
// FP32, so the descriptor inputs carry FP32 relative precision at any
// distance from the origin.
__device__ __forceinline__ void env_append(Env& E, bool valid, int slot, int j, double dxd, double dyd, double dzd,
                                           int elem, int& nR, int& nA, int (&nAs)[4], int& over)
{
    float r = 0.0f;
    bool inR = false, inA = false;
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) {
        const float dx = (float)dxd, dy = (float)dyd, dz = (float)dzd;
        r = sqrtf(dx * dx + dy * dy + dz * dz);
        inR = r < kCutRad;
        inA = r < kCutAng;
        const float inv = 1.0f / r;
        g = make_float4(dx * inv, dy * inv, dz * inv, r);
    }
    const unsigned long long mR = __ballot(inR);
    const int iR = nR + lanes_below(mR);
    // an angular entry refers to its radial entry: past the radial capacity
    // (an overflow, reported) the neighbour is left out of both sets, so that
    // every angular entry counted is one that was written
    const bool keepA = inA && iR < kRadMax;
    const unsigned long long mA = __ballot(keepA);
    const int iA = nA + lanes_below(mA);
    if (inR && iR < kRadMax) {
        E.geo[iR] = g;
        E.nid[iR] = j;
        const float x = r * (1.0f / kCutRad);
        E.fcr[iR] = make_float2(0.5f * cospif(x) + 0.5f, -0.5f * (kPi / kCutRad) * sinpif(x));
        E.info[iR] = (unsigned short)(elem | (slot << 2));
        if (inA && iA < kAngMax) {
            const float y = r * (1.0f / kCutAng);
            E.ang[iA] = (unsigned char)iR;
            E.afc[iA] = make_float2(0.5f * cospif(y) + 0.5f, -0.5f * (kPi / kCutAng) * sinpif(y));
        }
    }
#pragma unroll
    for (int e = 0; e < kNumSpecies; ++e) nAs[e] += __popcll(__ballot(keepA && elem == e));
    nR += __popcll(mR);
    nA += __popcll(mA);
    over |= (nR > kRadMax) | (nA > kAngMax);
}

__device__ __forceinline__ void env_finish(const Sys& S, Env& E, int nR, int nA, const int (&nAs)[4], int nS,
                                           int over)
{
    if (lane_id() == 0) {
        E.nR = nR < kRadMax ? nR : kRadMax;
        E.nA = nA < kAngMax ? nA : kAngMax;
        E.nS = nS;
        int acc = 0;
        for (int e = 0; e < kNumSpecies; ++e) {
            E.aseg[e] = acc < E.nA ? acc : E.nA;
            acc += nAs[e];
        }
        E.aseg[kNumSpecies] = E.nA;
        if (over) atomicOr(&S.st->overflow, 1);
        // observability maxima: touch the shared counters only when exceeded
        // (a plain read first keeps same-address atomics rare)
        StepState* st = S.st;
        if (nS > __hip_atomic_load(&st->max_ns, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&st->max_ns, nS);
        if (nR > __hip_atomic_load(&st->max_nr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&st->max_nr, nR);
        if (nA > __hip_atomic_load(&st->max_na, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&st->max_na, nA);
    }
    wave_sync();
}

// Candidate chunks of 64 atoms whose positions are loaded together before any
// of them is tested (the scan is bound by load latency, not arithmetic).
constexpr int kScanUnroll = 4;

// Pair-list test of a displacement (nearest image), with the same rounding
// wherever a list is built from a candidate scan.
__device__ __forceinline__ bool in_pair_list(const Sys& S, double dx, double dy, double dz)
{
    min_image(S, dx, dy, dz);
    return fma(dz, dz, fma(dy, dy, dx * dx)) < (double)S.rlist2;
}

// Builds only the pair list.
__device__ __forceinline__ void build_list(const Sys& S, int a)
{
    const int lane = lane_id();
    const double4 pa = S.pos[a];
    const int m = S.mol[a];
    int count = 0;
    const size_t base = (size_t)a * S.cap;
    for (int e = 0; e < kNumSpecies; ++e) {
        const int2 rg = S.mrange[m * kNumSpecies + e];
        for (int c0 = rg.x; c0 < rg.y; c0 += 64 * kScanUnroll) {
            double4 pc[kScanUnroll];
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                const int c = c0 + 64 * u + lane;
                if (c < rg.y) pc[u] = S.pos[c];
            }
#pragma unroll
            for (int u = 0; u < kScanUnroll; ++u) {
                if (c0 + 64 * u >= rg.y) break;  // wave-uniform
                const int c = c0 + 64 * u + lane;
                const bool ok = c < rg.y && c != a && in_pair_list(S, pc[u].x - pa.x, pc[u].y - pa.y, pc[u].z - pa.z);
                const unsigned long long mk = __ballot(ok);
                const int slot = count + lanes_below(mk);
                if (ok && slot < S.cap) S.nbr[base + slot] = c;
                count += __popcll(mk);
            }
        }
    }
    if (lane == 0) {
        S.ncnt[a] = count < S.cap ? count : S.cap;
        S.ref[a] = make_float4((float)pa.x, (float)pa.y, (float)pa.z, 0.f);
        if (count > S.cap) atomicOr(&S.st->overflow, 1);
    }
}

// Pair-list rebuild shared by the atoms of a tile when they all belong to one
// molecule scanned without a cell grid.  The workgroup reads each of the
// molecule's atoms once and applies build_list's test against every atom of
// the tile, keeping, in ascending index order, the atoms that pass for at
// least one of them with a mask of those it passes for; each atom's wave
// then writes its list from the kept atoms that carry its bit: the same
// candidates, tested by the same function in the same order, as build_list.
constexpr int kScanRoundsMax = 4;  // candidates per thread: CAP / NT (4096 / 1024 or 2048 / 512)

template <int CAP>
struct SharedScanT {
    int idx[CAP];        // kept atoms, ascending
    unsigned mask[CAP];  // bit i: within the list radius of tile atom i
    double tx[kTileCap], ty[kTileCap], tz[kTileCap];
    int ta[kTileCap], tm[kTileCap];  // tile atoms and their molecules
    int wcnt[kScanRoundsMax][16];    // kept atoms per (round, wave)
};
using SharedScan = SharedScanT<kSharedScanCap>;

// Candidate capacity of the shared scan of an NT-thread workgroup.
template <int NT>
constexpr int kScanCap = NT >= 1024 ? kSharedScanCap : kSharedScanCap / 2;

// Number of kept atoms, or -1 (nothing kept, workgroup-uniform) when the
// tile has no shared-scan molecule m (S.tile_mol) or its atoms turn out not
// to match it.  All threads of the workgroup call it.  The tile's molecule
// comes from the host's table, so the molecule's ranges and the candidates'
// positions are requested without waiting for the tile atoms' molecules,
// which are only checked; three barriers in all.
template <int NT, int CAP = kScanCap<NT>>
__device__ __forceinline__ int shared_scan(const Sys& S, int m, const int* atoms, int cnt, SharedScanT<CAP>& sc,
                                           int tid)
{
    constexpr int kRounds = CAP / NT;
    static_assert(kRounds * NT == CAP && kRounds <= kScanRoundsMax && NT / 64 <= 16, "candidates per thread");
    if (m < 0) return -1;
    int2 rg[kNumSpecies];
    int cum[kNumSpecies + 1];
    cum[0] = 0;
#pragma unroll
    for (int e = 0; e < kNumSpecies; ++e) {
        rg[e] = S.mrange[m * kNumSpecies + e];
        cum[e + 1] = cum[e] + (rg[e].y - rg[e].x);
    }
    // a molecule with a cell grid or more candidates than CAP is scanned by
    // each atom: decided (workgroup-uniformly) before anything is written
    if (S.molgrid[m] >= 0 || cum[kNumSpecies] > CAP) return -1;
    const int total = cum[kNumSpecies];
    // every position this thread tests is requested before any is tested
    double4 pc[kRounds];
    int cc[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int q = r * NT + tid;
        cc[r] = -1;
        pc[r] = make_double4(0.0, 0.0, 0.0, 0.0);
        if (q < total) {
            int c = 0;
#pragma unroll
            for (int e = 0; e < kNumSpecies; ++e)
                if (q >= cum[e] && q < cum[e + 1]) c = rg[e].x + (q - cum[e]);
            cc[r] = c;
            pc[r] = S.pos[c];
        }
    }
    if (tid < cnt) {
        const int a = atoms[tid];
        const double4 p = S.pos[a];
        sc.tx[tid] = p.x;
        sc.ty[tid] = p.y;
        sc.tz[tid] = p.z;
        sc.ta[tid] = a;
        sc.tm[tid] = S.mol[a];
    }
    __syncthreads();
    bool ok = true;
    for (int i = 0; i < cnt; ++i) ok = ok && sc.tm[i] == m;
    if (!ok) {  // workgroup-uniform; the barrier lets every thread finish reading tm
        __syncthreads();
        return -1;
    }
    const int wave = tid >> 6;
    unsigned mk[kRounds];
    unsigned long long bal[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        mk[r] = 0;
        if (cc[r] >= 0)
            for (int i = 0; i < cnt; ++i)
                if (cc[r] != sc.ta[i] &&
                    in_pair_list(S, pc[r].x - sc.tx[i], pc[r].y - sc.ty[i], pc[r].z - sc.tz[i]))
                    mk[r] |= 1u << i;
        bal[r] = __ballot(mk[r] != 0);
        if ((tid & 63) == 0) sc.wcnt[r][wave] = __popcll(bal[r]);
    }
    __syncthreads();
    int nl = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        int off = nl, tot = 0;
        for (int w = 0; w < NT / 64; ++w) {
            if (w < wave) off += sc.wcnt[r][w];
            tot += sc.wcnt[r][w];
        }
        if (mk[r] != 0) {
            const int slot = off + lanes_below(bal[r]);
            sc.idx[slot] = cc[r];
            sc.mask[slot] = mk[r];
        }
        nl += tot;
    }
    __syncthreads();
    return nl;
}

// Pair list of atom a, column `bit` of its tile, from the atoms kept by
// shared_scan.
template <int CAP>
__device__ __forceinline__ void build_list_shared(const Sys& S, int a, int bit, const SharedScanT<CAP>& sc, int nl)
{
    const int lane = lane_id();
    int count = 0;
    const size_t base = (size_t)a * S.cap;
    for (int s0 = 0; s0 < nl; s0 += 64) {
        const int s = s0 + lane;
        const bool ok = s < nl && ((sc.mask[s] >> bit) & 1u);
        const unsigned long long mk = __ballot(ok);
        const int slot = count + lanes_below(mk);
        if (ok && slot < S.cap) S.nbr[base + slot] = sc.idx[s];
        count += __popcll(mk);
    }
    if (lane == 0) {
        S.ncnt[a] = count < S.cap ? count : S.cap;
        S.ref[a] = make_float4((float)sc.tx[bit], (float)sc.ty[bit], (float)sc.tz[bit], 0.f);
        if (count > S.cap) atomicOr(&S.st->overflow, 1);
    }
}

// Loads the environment of atom a from its existing pair list.
__device__ __forceinline__ void load_env(const Sys& S, int a, Env& E)
{
    const int lane = lane_id();
    const double4 pa = S.pos[a];
    const int nS = S.ncnt[a];
    const size_t base = (size_t)a * S.cap;
    int nR = 0, nA = 0, over = 0;
    int nAs[4] = {0, 0, 0, 0};
    for (int s0 = 0; s0 < nS; s0 += 64) {
        const int s = s0 + lane;
        const bool valid = s < nS;
        double dx = 0, dy = 0, dz = 0;
        int elem = 0, j = 0;
        if (valid) {
            j = S.nbr[base + s];
            const double4 pj = S.pos[j];
            dx = pj.x - pa.x;
            dy = pj.y - pa.y;
            dz = pj.z - pa.z;
            min_image(S, dx, dy, dz);
            elem = (int)pj.w;
        }
        env_append(E, valid, s, j, dx, dy, dz, elem, nR, nA, nAs, over);
    }
    env_finish(S, E, nR, nA, nAs, nS, over);
}

// Rebuilds the pair list of atom a (all atoms of its molecule closer than
// 5.2 + skin, ascending index), then fills its environment from the new list:
// the cutoff functions are evaluated once per neighbour, not once per
// scanned chunk.  The fence makes the list written by the wave's lanes
// visible to all of them.
__device__ __forceinline__ void build_list_env(const Sys& S, int a, Env& E)
{
    build_list(S, a);
    __threadfence_block();
    load_env(S, a, E);
}

// Radial features G[0..63] of the wave's atom.  Lane (k, q): Gaussian k,
// neighbour subset q of 4; per-element sums, then a reduction over q.
__device__ __forceinline__ void radial_features(const Env& E, float* G)
{
    const int lane = lane_id();
    const int k = lane & 15, q = lane >> 4;
    const float Rk = 0.9f + 0.28f * (float)k;
    const int nR = E.nR;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int e = q; e < nR; e += 4) {
        const float r = E.geo[e].w;
        const float x = r - Rk;
        const float v = __expf(-kEtaRad * x * x) * E.fcr[e].x;
        const int s = E.info[e] & 3;
        a0 += s == 0 ? v : 0.f;
        a1 += s == 1 ? v : 0.f;
        a2 += s == 2 ? v : 0.f;
        a3 += s == 3 ? v : 0.f;
    }
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
        a0 += __shfl_xor(a0, off);
        a1 += __shfl_xor(a1, off);
        a2 += __shfl_xor(a2, off);
        a3 += __shfl_xor(a3, off);
    }
    if (q == 0) {
        G[k] = a0;
        G[16 + k] = a1;
        G[32 + k] = a2;
        G[48 + k] = a3;
    }
}

// Pair q (0 <= q < m (m-1)/2) -> (j < k), enumerated by k then j.
__device__ __forceinline__ void pair_of(int q, int& j, int& k)
{
    int kk = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)q)) * 0.5f);
    while (kk * (kk - 1) / 2 > q) --kk;
    while ((kk + 1) * kk / 2 <= q) ++kk;
    k = kk;
    j = q - kk * (kk - 1) / 2;
}

// Element pairs in feature-block order HH HC HN HO CC CN CO NN NO OO.
__constant__ static const unsigned char kPairS1[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
__constant__ static const unsigned char kPairS2[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
constexpr int kAccStride = 33;  // padded element-pair block of the angular accumulator

// The pairs (j < k) of angular neighbours of one atom, grouped by element
// pair p: j in the angular segment of element s1(p), k in that of s2(p).
// Every group is cut into runs of at most C consecutive pairs, C chosen so
// that all runs fit in the 64 lanes; a lane owns one run, so every pair it
// visits belongs to the same feature block.
struct PairRun {
    int p;            // element pair of the run, -1 when the lane has none
    int left;         // pairs in the run
    int jj, kk;       // position inside the group
    int lo1, lo2, n2; // segment starts, size of the second segment
    bool same;        // s1 == s2 (triangular group)
};

__device__ __forceinline__ PairRun lane_run(const Env& E, int lane)
{
    int seg[5];
#pragma unroll
    for (int e = 0; e < 5; ++e) seg[e] = E.aseg[e];
    int cnt[10], total = 0;
#pragma unroll
    for (int p = 0; p < 10; ++p) {
        const int s1 = kPairS1[p], s2 = kPairS2[p];
        const int n1 = seg[s1 + 1] - seg[s1], n2 = seg[s2 + 1] - seg[s2];
        cnt[p] = s1 == s2 ? n1 * (n1 - 1) / 2 : n1 * n2;
        total += cnt[p];
    }
    // run length C: ceil(total / 64) when its runs fit in the 64 lanes (every
    // lane busy), else max(that + 1, ceil(total / 54)), for which
    // sum_p ceil(cnt_p / C) < total / C + 10 <= 64 always holds.  Ceilings
    // use a float reciprocal with an exact integer correction.
    int C = total > 64 ? (total + 63) >> 6 : 1;
    int runs[10];
    for (int attempt = 0; attempt < 2; ++attempt) {
        const float inv = __builtin_amdgcn_rcpf((float)C);
        int sum = 0;
#pragma unroll
        for (int p = 0; p < 10; ++p) {
            int r = (int)((float)cnt[p] * inv + 0.5f);
            r += (r * C < cnt[p]) - ((r - 1) * C >= cnt[p] && r > 0);
            runs[p] = r;
            sum += r;
        }
        if (sum <= 64) break;
        int c54 = (int)((float)total * (1.0f / 54.0f) + 0.5f);
        c54 += (c54 * 54 < total) - ((c54 - 1) * 54 >= total && c54 > 0);
        C = max(C + 1, c54);
    }
    PairRun R;
    R.p = -1;
    R.left = 0;
    int first = 0, q0 = 0;
#pragma unroll
    for (int p = 0; p < 10; ++p) {
        if (lane >= first && lane < first + runs[p]) {
            const int s1 = kPairS1[p], s2 = kPairS2[p];
            q0 = (lane - first) * C;
            R.p = p;
            R.left = min(C, cnt[p] - q0);
            R.lo1 = seg[s1];
            R.lo2 = seg[s2];
            R.n2 = seg[s2 + 1] - seg[s2];
            R.same = s1 == s2;
        }
        first += runs[p];
    }
    if (R.p >= 0) {
        if (R.same) {
            pair_of(q0, R.jj, R.kk);
        } else {
            // q0 = jj * n2 + kk without an integer division
            int jj = (int)((float)q0 / (float)R.n2);
            while (jj * R.n2 > q0) --jj;
            while ((jj + 1) * R.n2 <= q0) ++jj;
            R.jj = jj;
            R.kk = q0 - jj * R.n2;
        }
    }
    return R;
}

// A run walks its pairs with one index fixed for several steps: k in a
// triangular group (pairs enumerated by k, then j < k), j otherwise.  x is
// that slowly changing index, y the one that moves every step; the terms are
// symmetric in the two neighbours, so (x, y) stands for (j, k) or (k, j).
__device__ __forceinline__ int run_x(const PairRun& R) { return R.same ? R.lo1 + R.kk : R.lo1 + R.jj; }
__device__ __forceinline__ int run_y(const PairRun& R) { return R.same ? R.lo1 + R.jj : R.lo2 + R.kk; }

// Advances to the next pair; true when x changed.
__device__ __forceinline__ bool run_next(PairRun& R)
{
    if (R.same) {
        if (++R.jj == R.kk) {
            ++R.kk;
            R.jj = 0;
            return true;
        }
        return false;
    }
    if (++R.kk == R.n2) {
        R.kk = 0;
        ++R.jj;
        return true;
    }
    return false;
}

// Value of lane (lane - d) of the same row of 16 lanes, 0 for the first d
// lanes of a row (DPP row shift).
template <int D>
__device__ __forceinline__ float row_shr(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x110 | D, 0xF, 0xF, false));
}

template <int D>
__device__ __forceinline__ float same_group_shr(int p)
{
    const int q = __builtin_amdgcn_update_dpp(-2, p, 0x110 | D, 0xF, 0xF, false);
    return (q == p && p >= 0) ? 1.f : 0.f;
}

// Adds the 32 angular terms of the pairs of run R (atom environment E) to t.
// The neighbours of the next pair are read from LDS before the terms of the
// current one are computed (their latency overlaps the arithmetic).
__device__ __forceinline__ void run_angular_terms(const Env& E, PairRun R, float (&t)[32])
{
    if (R.p < 0) return;
    float4 gx = E.geo[E.ang[run_x(R)]];
    float fx = E.afc[run_x(R)].x;
    float4 gy = E.geo[E.ang[run_y(R)]];
    float fy = E.afc[run_y(R)].x;
    for (int it = 0; it < R.left; ++it) {
        const bool more = it + 1 < R.left;
        const bool xc = run_next(R);
        float4 gxn = gx, gyn = gy;
        float fxn = fx, fyn = fy;
        if (more) {
            const int y = run_y(R);
            gyn = E.geo[E.ang[y]];
            fyn = E.afc[y].x;
            if (xc) {
                const int x = run_x(R);
                gxn = E.geo[E.ang[x]];
                fxn = E.afc[x].x;
            }
        }
        const float c = gx.x * gy.x + gx.y * gy.y + gx.z * gy.z;
        const float cp = kCosScale * c;
        const float sp = __builtin_amdgcn_sqrtf(fmaxf(0.f, 1.f - cp * cp));
        const float w = kTwoPowM31 * fx * fy;
        const float rbar = 0.5f * (gx.w + gy.w);
        float B[kNumShells];
#pragma unroll
        for (int m = 0; m < kNumShells; ++m) {
            const float x = rbar - (0.9f + 0.65f * (float)m);
            B[m] = w * __expf(-kEtaAng * x * x);
        }
#pragma unroll
        for (int n = 0; n < kNumSectors; ++n) {
            float u = 1.f + cp * kSecCos[n] + sp * kSecSin[n];
            u = u * u;  // ^2
            u = u * u;  // ^4
            u = u * u;  // ^8
            u = u * u;  // ^16
            u = u * u;  // ^32
#pragma unroll
            for (int m = 0; m < kNumShells; ++m) t[8 * m + n] += u * B[m];
        }
        gx = gxn;
        fx = fxn;
        gy = gyn;
        fy = fyn;
    }
}

// Segmented inclusive scan of the 32 values of t inside each row of 16
// lanes (DPP shifts 1, 2, 4, 8) over runs of equal key; returns true in the
// last lane of each (row, key) segment, which then holds the segment's sums.
// Lanes with key < 0 take no part.  All 64 lanes must execute it.
__device__ __forceinline__ bool row_segment_sums(int key, float (&t)[32])
{
    const float m1 = same_group_shr<1>(key), m2 = same_group_shr<2>(key);
    const float m4 = same_group_shr<4>(key), m8 = same_group_shr<8>(key);
    const int kn = __builtin_amdgcn_update_dpp(-3, key, 0x101, 0xF, 0xF, false);  // lane + 1 of the row
#pragma unroll
    for (int f = 0; f < 32; ++f) {
        float v = t[f];
        v = fmaf(m1, row_shr<1>(v), v);
        v = fmaf(m2, row_shr<2>(v), v);
        v = fmaf(m4, row_shr<4>(v), v);
        v = fmaf(m8, row_shr<8>(v), v);
        t[f] = v;
    }
    return key >= 0 && kn != key;
}

// Angular features of the wave's atom, accumulated into acc[10][33] (LDS,
// zeroed beforehand).  Each lane sums the 32 terms of its run in registers;
// runs of one element pair occupy consecutive lanes, so a segmented scan
// inside each row of 16 lanes leaves every (row, element pair) total in the
// last lane of its segment, and only those lanes add to LDS (one
// instruction per feature: a fixed order).  Element-pair blocks 33 floats
// apart sit in different banks.  The caller copies acc into G[64 + 32 p + f].
__device__ __forceinline__ void angular_features(const Env& E, float* acc)
{
    const int lane = lane_id();
    const PairRun R = lane_run(E, lane);
    float t[32];
#pragma unroll
    for (int f = 0; f < 32; ++f) t[f] = 0.f;
    run_angular_terms(E, R, t);
    if (row_segment_sums(R.p, t)) {
        float* dst = acc + kAccStride * R.p;
#pragma unroll
        for (int f = 0; f < 32; ++f) atomicAdd(dst + f, t[f]);
    }
}

// G[64..383] <- acc[10][33] (wave-cooperative; acc complete).
__device__ __forceinline__ void angular_store(const float* acc, float* G)
{
    const int lane = lane_id();
    for (int i = lane; i < 320; i += 64) G[64 + i] = acc[kAccStride * (i >> 5) + (i & 31)];
}

// Adjoint of the descriptors for the wave's atom a: given g = dE_a/dG_a
// (LDS), accumulates the force on every neighbour within 5.2 A due to E_a into
// facc[3 * entry] (LDS).  Radial entries are owned by one lane each (plain
// store); the angular pairs then add with LDS atomics.  The caller separates
// the two phases with a barrier.
// Force on radial entry e of the atom from its radial features: g holds
// the atom's dE/dG radial part (16 values per neighbour element).
__device__ __forceinline__ float3 radial_force(const Env& E, int e, const float* g)
{
    const float4 ge = E.geo[e];
    const float2 f = E.fcr[e];
    const float* gs = g + 16 * (E.info[e] & 3);
    float dEdr = 0.f;
#pragma unroll
    for (int k = 0; k < kNumRadial; ++k) {
        const float x = ge.w - (0.9f + 0.28f * (float)k);
        const float ex = __expf(-kEtaRad * x * x);
        dEdr += gs[k] * ex * (f.y - 2.f * kEtaRad * x * f.x);
    }
    return make_float3(-dEdr * ge.x, -dEdr * ge.y, -dEdr * ge.z);
}

__device__ __forceinline__ void adjoint_radial(const Env& E, const float* g, float* facc)
{
    const int lane = lane_id();
    const int nR = E.nR;
    for (int e = lane; e < nR; e += 64) {
        const float3 v = radial_force(E, e, g);
        facc[3 * e + 0] = v.x;
        facc[3 * e + 1] = v.y;
        facc[3 * e + 2] = v.z;
    }
}

// Adjoint of the angular terms of run R: with gm the 32 values of dE/dG of
// the run's element-pair block, add(radial entry, angular entry, v) receives
// the gradient v of E_a with respect to the position of that neighbour (the
// force is -v).  The slowly changing neighbour x is summed in registers and
// handed over when x changes; y at every pair.
template <class Add>
__device__ __forceinline__ void adjoint_run(const Env& E, PairRun R, const float (&gm)[32], Add add)
{
    if (R.p < 0) return;
    int xa = run_x(R), ya = run_y(R);
    int ex = E.ang[xa], ey = E.ang[ya];
    float4 gx = E.geo[ex], gy = E.geo[ey];
    float2 fx = E.afc[xa], fy = E.afc[ya];
    float ax = 0.f, ay = 0.f, az = 0.f;
    for (int it = 0; it < R.left; ++it) {
        // next pair's neighbours first (see run_angular_terms)
        const bool more = it + 1 < R.left;
        const bool xc = run_next(R) && more;
        int xan = xa, yan = ya, exn = ex, eyn = ey;
        float4 gxn = gx, gyn = gy;
        float2 fxn = fx, fyn = fy;
        if (more) {
            yan = run_y(R);
            eyn = E.ang[yan];
            gyn = E.geo[eyn];
            fyn = E.afc[yan];
            if (xc) {
                xan = run_x(R);
                exn = E.ang[xan];
                gxn = E.geo[exn];
                fxn = E.afc[xan];
            }
        }
        const float c = gx.x * gy.x + gx.y * gy.y + gx.z * gy.z;
        const float cp = kCosScale * c;
        const float sp = __builtin_amdgcn_sqrtf(fmaxf(0.f, 1.f - cp * cp));
        const float rbar = 0.5f * (gx.w + gy.w);
        // P_n = sum_m g_mn B_m, Q_n = sum_m g_mn dB_m/drbar
        float P[kNumSectors], Q[kNumSectors];
#pragma unroll
        for (int n = 0; n < kNumSectors; ++n) {
            P[n] = 0.f;
            Q[n] = 0.f;
        }
#pragma unroll
        for (int m = 0; m < kNumShells; ++m) {
            const float x = rbar - (0.9f + 0.65f * (float)m);
            const float Bm = __expf(-kEtaAng * x * x);
            const float dBm = -2.f * kEtaAng * x * Bm;
#pragma unroll
            for (int n = 0; n < kNumSectors; ++n) {
                P[n] += gm[8 * m + n] * Bm;
                Q[n] += gm[8 * m + n] * dBm;
            }
        }
        float Et = 0.f, dEdcp = 0.f, dEdrb = 0.f;
        const float inv_sp = __builtin_amdgcn_rcpf(sp);  // sp >= sqrt(1 - 0.95^2)
#pragma unroll
        for (int n = 0; n < kNumSectors; ++n) {
            const float ct = kSecCos[n], st = kSecSin[n];
            const float u = 1.f + cp * ct + sp * st;
            const float u2 = u * u, u4 = u2 * u2, u8 = u4 * u4, u16 = u8 * u8;
            const float u31 = u16 * u8 * u4 * u2 * u;
            const float A = u31 * u;
            const float dA = 32.f * u31 * (ct - cp * st * inv_sp);
            Et += A * P[n];
            dEdcp += dA * P[n];
            dEdrb += A * Q[n];
        }
        // E_t = w * sum_n A_n P_n with w = 2^-31 fc_x fc_y
        const float pre = kTwoPowM31;
        const float ff = fx.x * fy.x;
        const float dEdc = pre * ff * kCosScale * dEdcp;
        const float dEdrx = pre * (Et * fx.y * fy.x + 0.5f * ff * dEdrb);
        const float dEdry = pre * (Et * fx.x * fy.y + 0.5f * ff * dEdrb);
        const float ix = __builtin_amdgcn_rcpf(gx.w), iy = __builtin_amdgcn_rcpf(gy.w);
        ax += dEdrx * gx.x + dEdc * (gy.x - c * gx.x) * ix;
        ay += dEdrx * gx.y + dEdc * (gy.y - c * gx.y) * ix;
        az += dEdrx * gx.z + dEdc * (gy.z - c * gx.z) * ix;
        add(ey, ya, dEdry * gy.x + dEdc * (gx.x - c * gy.x) * iy, dEdry * gy.y + dEdc * (gx.y - c * gy.y) * iy,
            dEdry * gy.z + dEdc * (gx.z - c * gy.z) * iy);
        if (xc) {
            add(ex, xa, ax, ay, az);
            ax = ay = az = 0.f;
        }
        xa = xan;
        ya = yan;
        ex = exn;
        ey = eyn;
        gx = gxn;
        gy = gyn;
        fx = fxn;
        fy = fyn;
    }
    add(ex, xa, ax, ay, az);
}

// dE/dG values of element-pair block p of a G row, held in registers.
__device__ __forceinline__ void load_block(const float* g, int p, float (&gm)[32])
{
    const float4* gb = reinterpret_cast<const float4*>(g + 64 + 32 * p);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float4 v = gb[q];
        gm[4 * q + 0] = v.x;
        gm[4 * q + 1] = v.y;
        gm[4 * q + 2] = v.z;
        gm[4 * q + 3] = v.w;
    }
}

// Angular part of the adjoint for the wave's atom: forces added to facc
// with LDS atomics (one wave per atom, so each address sees the adds of one
// wave only).
__device__ __forceinline__ void adjoint_angular(const Env& E, const float* g, float* facc)
{
    const PairRun R = lane_run(E, lane_id());
    if (R.p < 0) return;
    float gm[32];
    load_block(g, R.p, gm);
    adjoint_run(E, R, gm, [&](int e, int, float vx, float vy, float vz) {
        atomicAdd(&facc[3 * e + 0], -vx);
        atomicAdd(&facc[3 * e + 1], -vy);
        atomicAdd(&facc[3 * e + 2], -vz);
    });
}

// Fixed-point force of one neighbour entry (kFixScale units), or false when
// a component is not finite or beyond kFixMax.
__device__ __forceinline__ bool fixed_vec(float fx, float fy, float fz, long long& qx, long long& qy, long long& qz)
{
    if (!(fabsf(fx) < kFixMax && fabsf(fy) < kFixMax && fabsf(fz) < kFixMax)) return false;
    qx = __double2ll_rn((double)fx * kFixScale);
    qy = __double2ll_rn((double)fy * kFixScale);
    qz = __double2ll_rn((double)fz * kFixScale);
    return true;
}

__device__ __forceinline__ bool fixed_force(const float* facc, int e, long long& qx, long long& qy, long long& qz)
{
    return fixed_vec(facc[3 * e], facc[3 * e + 1], facc[3 * e + 2], qx, qy, qz);
}

__device__ __forceinline__ void global_force_add(const Sys& S, int j, long long qx, long long qy, long long qz)
{
    unsigned long long* fj = S.facc + 4 * (size_t)j;
    atomicAdd(fj + 0, (unsigned long long)qx);
    atomicAdd(fj + 1, (unsigned long long)qy);
    atomicAdd(fj + 2, (unsigned long long)qz);
}

// Workgroup table that merges the force contributions of a tile's atoms per
// receiving atom before they go to HBM (the atoms of a tile are spatial
// neighbours and share most of their neighbours).  Open addressing over nh
// slots: key = atom index (-1 empty), three fixed-point sums.
struct ForceTable {
    int* key;
    long long* v;  // [3][nh]
    int nh;
};

__device__ __forceinline__ ForceTable force_table(void* mem, size_t bytes)
{
    ForceTable t;
    t.nh = (int)(bytes / (sizeof(int) + 3 * sizeof(long long))) & ~1;
    t.v = reinterpret_cast<long long*>(mem);
    t.key = reinterpret_cast<int*>(t.v + 3 * (size_t)t.nh);
    return t;
}

__device__ __forceinline__ void table_clear(const ForceTable& t, int tid, int nthr)
{
    for (int i = tid; i < t.nh; i += nthr) {
        t.key[i] = -1;
        t.v[i] = 0;
        t.v[t.nh + i] = 0;
        t.v[2 * t.nh + i] = 0;
    }
}

constexpr int kTableProbes = 32;

// Adds (qx, qy, qz) for atom j to the table; past kTableProbes occupied
// slots it goes straight to HBM.  Integer sums: the result does not depend
// on the order of the adds.
__device__ __forceinline__ void table_add(const Sys& S, const ForceTable& t, int j, long long qx, long long qy,
                                          long long qz)
{
    unsigned h = (unsigned)(((unsigned long long)((unsigned)j * 0x9E3779B1u) * (unsigned)t.nh) >> 32);
    for (int probe = 0; probe < kTableProbes; ++probe) {
        int k = t.key[h];
        if (k == -1) k = atomicCAS(&t.key[h], -1, j);
        if (k == -1 || k == j) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&t.v[h]), (unsigned long long)qx);
            atomicAdd(reinterpret_cast<unsigned long long*>(&t.v[t.nh + h]), (unsigned long long)qy);
            atomicAdd(reinterpret_cast<unsigned long long*>(&t.v[2 * t.nh + h]), (unsigned long long)qz);
            return;
        }
        h = h + 1 == (unsigned)t.nh ? 0u : h + 1;
    }
    global_force_add(S, j, qx, qy, qz);
}

// Forces of E_a for the wave's atom a: each neighbour within 5.2 A receives
// its force (LDS facc[3 * entry]), a receives minus their sum (translation
// invariance of E_a).  Components are rounded to multiples of 2^-32 eV/A
// once per neighbour.  A non-finite component or one beyond kFixMax sets
// the non-finite flag instead of being added.
__device__ __forceinline__ void table_add_atom(const Sys& S, const ForceTable& t, int a, const Env& E,
                                               const float* facc)
{
    const int lane = lane_id();
    long long sx = 0, sy = 0, sz = 0;
    bool bad = false;
    for (int e = lane; e < E.nR; e += 64) {
        long long qx, qy, qz;
        if (!fixed_force(facc, e, qx, qy, qz)) {
            bad = true;
            continue;
        }
        table_add(S, t, E.nid[e], qx, qy, qz);
        sx += qx;
        sy += qy;
        sz += qz;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_xor(sx, off);
        sy += __shfl_xor(sy, off);
        sz += __shfl_xor(sz, off);
    }
    if (lane == 0) table_add(S, t, a, -sx, -sy, -sz);
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(&S.st->nonfinite, 1);
}

// Adds the table's sums to the HBM accumulators (workgroup-wide).
__device__ __forceinline__ void table_flush(const Sys& S, const ForceTable& t, int tid, int nthr)
{
    for (int i = tid; i < t.nh; i += nthr) {
        const int j = t.key[i];
        if (j >= 0) global_force_add(S, j, t.v[i], t.v[t.nh + i], t.v[2 * t.nh + i]);
    }
}

// LDS row strides (elements) of the activation buffers.
constexpr int kLdG = kNumFeat + 8;  // G / dE/dG rows: fp32, or bf16 hi + lo overlaid
constexpr int kLd1 = kH1 + 8;       // bf16 rows
constexpr int kLd2 = kH2 + 8;
constexpr int kLd3 = kH3 + 8;
constexpr int kLdF1 = kH1 + 4;      // fp32 rows
constexpr int kLdF2 = kH2 + 4;
constexpr int kLdF3 = kH3 + 4;

// ------------------------------------------------------------------------
// Angular work pooled over the workgroup.  The pairs of all atoms of a tile
// are dealt out to all its lanes in runs of one (atom, element pair) group,
// so the angular phases last as long as the tile's mean work instead of its
// heaviest atom's.  Sums that receive adds from several waves are kept in
// 64-bit fixed point (2^-32 units): integer addition does not depend on the
// order of the adds.
// ------------------------------------------------------------------------
template <int T>
struct PoolPlan {
    int cnt[T * 10];        // pairs of group g = 10 w + p (atom w, element pair p)
    int first[T * 10 + 1];  // first lane of each group's runs; first[10 T] = lanes used
    int C;                  // pairs per run
};

// Group sizes, run length and lane ranges for the first nact atoms of the
// tile, computed by one wave (lane: groups GPL lane .. GPL lane + GPL - 1)
// while the others do other work; the caller's next barrier publishes the
// plan.  C = ceil(W / (NT - 10 T)) for W pairs in all keeps the runs within
// the NT lanes of the workgroup: sum_g ceil(cnt_g / C) < W / C + 10 T <= NT.
template <int T, int NT>
__device__ __forceinline__ void pool_plan_wave(const Env* env, int nact, PoolPlan<T>& pl, int lane)
{
    constexpr int NG = T * 10, FREE = NT - NG, GPL = (NG + 63) / 64;
    static_assert(FREE > 0, "more lanes than groups");
    auto group_size = [&](int g) {
        if (g >= NG || g / 10 >= nact) return 0;  // no atom in this column of the tile
        const Env& E = env[g / 10];
        const int p = g % 10;
        const int s1 = kPairS1[p], s2 = kPairS2[p];
        const int n1 = E.aseg[s1 + 1] - E.aseg[s1], n2 = E.aseg[s2 + 1] - E.aseg[s2];
        return s1 == s2 ? n1 * (n1 - 1) / 2 : n1 * n2;
    };
    int c[GPL], w = 0;
#pragma unroll
    for (int i = 0; i < GPL; ++i) {
        c[i] = group_size(GPL * lane + i);
        w += c[i];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
    const int C = w > FREE ? (w + FREE - 1) / FREE : 1;
    int r[GPL], mine = 0;
#pragma unroll
    for (int i = 0; i < GPL; ++i) {
        r[i] = (c[i] + C - 1) / C;
        mine += r[i];
    }
    int incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    int at = incl - mine;
#pragma unroll
    for (int i = 0; i < GPL; ++i) {
        const int g = GPL * lane + i;
        if (g < NG) {
            pl.cnt[g] = c[i];
            pl.first[g] = at;
        }
        at += r[i];
    }
    if (lane == 63) pl.first[NG] = incl;
    if (lane == 0) pl.C = C;
}

// The (atom, element pair) group whose run workgroup lane L takes, or -1:
// the last group whose first lane is <= L (groups without runs share their
// successor's first lane).  A binary search of dependent LDS reads, so the
// fused kernel finds it once and keeps it for the adjoint.
template <int T>
__device__ __forceinline__ int pool_group(const PoolPlan<T>& pl, int L)
{
    constexpr int NG = T * 10;
    if (L >= pl.first[NG]) return -1;
    int lo = 0, hi = NG - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pl.first[mid] <= L)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The run of workgroup lane L in group g = pool_group(pl, L) (R.p < 0 when
// L has none); w = its atom.
template <int T>
__device__ __forceinline__ PairRun pool_run(const Env* env, const PoolPlan<T>& pl, int L, int g, int& w)
{
    PairRun R;
    R.p = -1;
    R.left = 0;
    w = 0;
    if (g < 0) return R;
    w = g / 10;
    const int p = g - 10 * w;
    const Env& E = env[w];
    const int q0 = (L - pl.first[g]) * pl.C;
    const int s1 = kPairS1[p], s2 = kPairS2[p];
    R.p = p;
    R.left = min(pl.C, pl.cnt[g] - q0);
    R.lo1 = E.aseg[s1];
    R.lo2 = E.aseg[s2];
    R.n2 = E.aseg[s2 + 1] - E.aseg[s2];
    R.same = s1 == s2;
    if (R.same) {
        pair_of(q0, R.jj, R.kk);
    } else {
        int jj = (int)((float)q0 / (float)R.n2);
        while (jj * R.n2 > q0) --jj;
        while ((jj + 1) * R.n2 <= q0) ++jj;
        R.jj = jj;
        R.kk = q0 - jj * R.n2;
    }
    return R;
}

// x >= 0 (a sum of non-negative terms) in 2^-32 units.
__device__ __forceinline__ unsigned long long to_fix_pos(float x)
{
    const float fl = floorf(x);
    const unsigned hi = (unsigned)fl;
    const unsigned lo = (unsigned)((x - fl) * 4294967296.0f);
    return ((unsigned long long)hi << 32) | lo;
}

// |x| < kFixMax in 2^-32 units (two's complement).
__device__ __forceinline__ long long to_fix(float x)
{
    const float fl = floorf(x);
    const int hi = (int)fl;
    const unsigned lo = (unsigned)((x - fl) * 4294967296.0f);
    return (long long)(((unsigned long long)(unsigned)hi << 32) | lo);
}

// Angular features of the tile's atoms: accI[w][32 p + f] (fixed point,
// zeroed beforehand) receives the row-segment sums (key = group).
template <int T>
__device__ __forceinline__ void angular_features_pooled(const Env* env, const PoolPlan<T>& pl,
                                                        unsigned long long* accI, int tid, int g)
{
    int w;
    const PairRun R = pool_run<T>(env, pl, tid, g, w);
    float t[32];
#pragma unroll
    for (int f = 0; f < 32; ++f) t[f] = 0.f;
    run_angular_terms(env[w], R, t);
    if (row_segment_sums(R.p >= 0 ? 10 * w + R.p : -1, t)) {
        unsigned long long* dst = accI + 320 * w + 32 * R.p;
#pragma unroll
        for (int f = 0; f < 32; ++f) atomicAdd(dst + f, to_fix_pos(t[f]));
    }
}

// G[w][64 + i] <- accI[w][i] (workgroup-wide).
template <int T>
__device__ __forceinline__ void angular_store_pooled(const unsigned long long* accI, float* G, int tid, int nthr)
{
    for (int i = tid; i < T * 320; i += nthr) {
        const int w = i / 320, f = i - 320 * w;
        G[w * kLdG + 64 + f] = (float)((double)accI[i] * (1.0 / 4294967296.0));
    }
}

// Angular part of the adjoint for the tile: faccA[(w kAngMax + j) 3 + c]
// (fixed point, zeroed beforehand) receives the force on angular entry j of
// atom w.  G holds the dE/dG rows.  bad: a component reached kFixMax.
template <int T>
__device__ __forceinline__ void adjoint_angular_pooled(const Sys& S, const Env* env, const PoolPlan<T>& pl,
                                                       const float* G, unsigned long long* faccA, int tid, int g)
{
    int w;
    const PairRun R = pool_run<T>(env, pl, tid, g, w);
    bool bad = false;
    if (R.p >= 0) {
        float gm[32];
        load_block(G + w * kLdG, R.p, gm);
        unsigned long long* fa = faccA + (size_t)w * kAngMax * 3;
        adjoint_run(env[w], R, gm, [&](int, int j, float vx, float vy, float vz) {
            if (!(fabsf(vx) < kFixMax && fabsf(vy) < kFixMax && fabsf(vz) < kFixMax)) {
                bad = true;
                return;
            }
            atomicAdd(fa + 3 * j + 0, (unsigned long long)to_fix(-vx));
            atomicAdd(fa + 3 * j + 1, (unsigned long long)to_fix(-vy));
            atomicAdd(fa + 3 * j + 2, (unsigned long long)to_fix(-vz));
        });
    }
    if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&S.st->nonfinite, 1);
}

// Forces of E_a for the wave's atom a, merged in the table: the radial part
// computed here from g (the atom's 64 radial dE/dG values), the pooled
// angular part from faccA (fixed point).
__device__ __forceinline__ void table_add_atom_pooled(const Sys& S, const ForceTable& t, int a, const Env& E,
                                                      const float* g, const unsigned long long* faccA)
{
    const int lane = lane_id();
    long long sx = 0, sy = 0, sz = 0;
    bool bad = false;
    // angular entries are the radial entries within the angular cutoff, in
    // radial order (env_append): entry e is angular entry j = the number of
    // such entries before it, so each neighbour takes one table add with its
    // radial and angular parts (integer sums: the same totals)
    int jbase = 0;
    for (int e0 = 0; e0 < E.nR; e0 += 64) {  // wave-uniform
        const int e = e0 + lane;
        const bool live = e < E.nR;
        const bool isA = live && E.geo[e].w < kCutAng;
        const unsigned long long mA = __ballot(isA);
        const int j = jbase + lanes_below(mA);
        jbase += __popcll(mA);
        if (!live) continue;
        long long qx, qy, qz;
        const float3 v = radial_force(E, e, g);
        if (!fixed_vec(v.x, v.y, v.z, qx, qy, qz)) {
            bad = true;
            continue;
        }
        if (isA && j < E.nA) {
            qx += (long long)faccA[3 * j];
            qy += (long long)faccA[3 * j + 1];
            qz += (long long)faccA[3 * j + 2];
        }
        table_add(S, t, E.nid[e], qx, qy, qz);
        sx += qx;
        sy += qy;
        sz += qz;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_xor(sx, off);
        sy += __shfl_xor(sy, off);
        sz += __shfl_xor(sz, off);
    }
    if (lane == 0) table_add(S, t, a, -sx, -sy, -sz);
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(&S.st->nonfinite, 1);
}

// ------------------------------------------------------------------------
// Network on a tile of up to T atoms of one element (workgroup-wide).
// ------------------------------------------------------------------------


// out[t][o] = sum_k in[t][k] * Wm[k][o] (+ epilogue) for o < M, t < T.
// Thread = (output o, group of 4 atoms).
template <int T, int K, int M, int EPI>
__device__ __forceinline__ void dense_f32(const float* in, int ldi, const float* __restrict__ Wm,
                                          const float* __restrict__ bias, float* out, int ldo, float* aux,
                                          int ldaux, int tid, int nthr)
{
    constexpr int NG = (T + 3) / 4;
    for (int idx = tid; idx < M * NG; idx += nthr) {
        const int o = idx % M, ag = idx / M;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int k = 0; k < K; k += 4) {
            const float w0 = Wm[(k + 0) * M + o], w1 = Wm[(k + 1) * M + o];
            const float w2 = Wm[(k + 2) * M + o], w3 = Wm[(k + 3) * M + o];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                // rows past T (T not a multiple of 4) re-read row T - 1; discarded below
                const int row = 4 * ag + t < T ? 4 * ag + t : T - 1;
                const float4 x = *reinterpret_cast<const float4*>(in + row * ldi + k);
                acc[t] += x.x * w0 + x.y * w1 + x.z * w2 + x.w * w3;
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int at = 4 * ag + t;
            if (at >= T) break;
            float v = acc[t];
            if (EPI == 0) {  // forward: z = v + b; out = celu(z); aux = celu'(z)
                const float z = v + bias[o];
                out[at * ldo + o] = celu_f(z);
                aux[at * ldaux + o] = celu_d(z);
            } else if (EPI == 1) {  // backward: out = v * aux
                out[at * ldo + o] = v * aux[at * ldaux + o];
            } else {  // plain store
                out[at * ldo + o] = v;
            }
        }
    }
}

// Per-tile LDS of the FP32 network (rows of T atoms).
template <int T>
struct MlpF32Smem {
    float h1[T * kLdF1], d1[T * kLdF1];
    float h2[T * kLdF2], d2[T * kLdF2];
    float h3[T * kLdF3], d3[T * kLdF3];
};

// FP32 network forward + input gradient on VALU.  G: [T][kLdG] fp32 in LDS,
// replaced by dE/dG when GRAD.  E[T] receives the atom energies.
template <int T, bool GRAD>
__device__ __forceinline__ void mlp_f32(const float* __restrict__ w, float* G, MlpF32Smem<T>& sm, float* E, int tid, int nthr)
{
    using L = W32Layout;
    dense_f32<T, kNumFeat, kH1, 0>(G, kLdG, w + L::Wt1, w + L::B1, sm.h1, kLdF1, sm.d1, kLdF1, tid, nthr);
    __syncthreads();
    dense_f32<T, kH1, kH2, 0>(sm.h1, kLdF1, w + L::Wt2, w + L::B2, sm.h2, kLdF2, sm.d2, kLdF2, tid, nthr);
    __syncthreads();
    dense_f32<T, kH2, kH3, 0>(sm.h2, kLdF2, w + L::Wt3, w + L::B3, sm.h3, kLdF3, sm.d3, kLdF3, tid, nthr);
    __syncthreads();
    // output layer: one wave per atom
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    for (int t = wave; t < T; t += nw) {
        float s = 0.f;
        for (int o = lane; o < kH3; o += 64) s += w[L::W4 + o] * sm.h3[t * kLdF3 + o];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) E[t] = s + w[L::B4];
    }
    if (!GRAD) return;
    // delta3 = celu'(z3) * W4, in place of d3
    for (int idx = tid; idx < T * kH3; idx += nthr) {
        const int t = idx / kH3, o = idx % kH3;
        sm.d3[t * kLdF3 + o] *= w[L::W4 + o];
    }
    __syncthreads();
    // delta2 = celu'(z2) * (W3^T delta3): W3 is [96][128] = [k][m]
    dense_f32<T, kH3, kH2, 1>(sm.d3, kLdF3, w + L::W3, nullptr, sm.h2, kLdF2, sm.d2, kLdF2, tid, nthr);
    __syncthreads();
    dense_f32<T, kH2, kH1, 1>(sm.h2, kLdF2, w + L::W2, nullptr, sm.h1, kLdF1, sm.d1, kLdF1, tid, nthr);
    __syncthreads();
    dense_f32<T, kH1, kNumFeat, 2>(sm.h1, kLdF1, w + L::W1, nullptr, G, kLdG, nullptr, 0, tid, nthr);
    __syncthreads();
}

// Per-tile LDS of the MFMA network.  Activations are stored as BF16 (and,
// in the split mode, a second BF16 array with the rounding residual), written
// once by the producing layer's epilogue and read as B operands by every
// output tile of the next layer.
template <int T, bool SPLIT>
struct MlpMfmaSmem {
    static constexpr int NL = SPLIT ? 2 : 1;  // hi, and lo when split
    __bf16 h1[NL][T * kLd1];  // h1, later delta1
    __bf16 h2[NL][T * kLd2];  // h2, later delta2
    __bf16 h3[NL][T * kLd3];  // delta3
    float d1[T * kLdF1];      // celu'(z1)
    float d2[T * kLdF2];      // celu'(z2)
    float ep[8 * 16];         // output-layer partial sums per (m tile, atom)
};

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

// Four consecutive activations (idx a multiple of 4): one 8-byte store per
// array.
template <bool SPLIT>
__device__ __forceinline__ void put_act4(__bf16* hi, __bf16* lo, int idx, const floatx4& v)
{
    bf16x4 h, l;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h[i] = (__bf16)v[i];
        if constexpr (SPLIT) l[i] = (__bf16)(v[i] - (float)h[i]);
    }
    *reinterpret_cast<bf16x4*>(hi + idx) = h;
    if constexpr (SPLIT) *reinterpret_cast<bf16x4*>(lo + idx) = l;
}

template <bool SPLIT>
__device__ __forceinline__ void put_act(__bf16* hi, __bf16* lo, int idx, float v)
{
    const __bf16 h = (__bf16)v;
    hi[idx] = h;
    if constexpr (SPLIT) lo[idx] = (__bf16)(v - (float)h);
}

// G (fp32 [T][kLdG], complete) -> bf16 hi (and lo) rows overlaid on the same
// LDS: hi at G, lo right after T rows of hi.  Workgroup-wide.
template <int T, bool SPLIT>
__device__ __forceinline__ void split_g_inplace(float* G, int tid, int nthr)
{
    constexpr int PER = (T * kNumFeat + 64 * T - 1) / (64 * T);
    float v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = tid + q * nthr;
        v[q] = i < T * kNumFeat ? G[(i / kNumFeat) * kLdG + i % kNumFeat] : 0.f;
    }
    __syncthreads();
    __bf16* hi = reinterpret_cast<__bf16*>(G);
    __bf16* lo = hi + T * kLdG;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = tid + q * nthr;
        if (i < T * kNumFeat) put_act<SPLIT>(hi, lo, (i / kNumFeat) * kLdG + i % kNumFeat, v[q]);
    }
    __syncthreads();
}

// One 16 x 16 output tile: rows = outputs of fragment row mt, columns =
// atoms (columns >= T are zero).  A from pre-swizzled weight fragments
// (HBM/L2), B from LDS rows.  SPLIT: D = A_hi B_hi + A_hi B_lo + A_lo B_hi
// (FP32 accumulation).
template <int T, int KT, bool SPLIT>
__device__ __forceinline__ floatx4 mfma_tile(const bf16x8* __restrict__ fhi, const bf16x8* __restrict__ flo,
                                             const __bf16* bhi, const __bf16* blo, int ld, int lane)
{
    // independent accumulators (hi*hi / hi*lo / lo*hi, or even / odd k
    // steps) keep several MFMAs in flight instead of one dependent chain
    floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0, acc2 = acc0;
    const int col = lane & 15, kq = (lane >> 4) * 8;
    const bool live = col < T;
    const bf16x8 zero = {};
    const int off = (live ? col : 0) * ld + kq;
    // a partial unroll bounds the fragments in flight (registers) in the
    // split mode, which reads twice the operands per step
#pragma unroll(SPLIT ? 4 : 6)
    for (int kt = 0; kt < KT; ++kt) {
        const bf16x8 a = fhi[kt * 64 + lane];
        bf16x8 bh = *reinterpret_cast<const bf16x8*>(bhi + off + kt * 32);
        if (!live) bh = zero;
        if constexpr (SPLIT) {
            bf16x8 bl = *reinterpret_cast<const bf16x8*>(blo + off + kt * 32);
            if (!live) bl = zero;
            const bf16x8 al = flo[kt * 64 + lane];
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc2, 0, 0, 0);
        } else if (kt & 1) {
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc1, 0, 0, 0);
        } else {
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc0, 0, 0, 0);
        }
    }
    floatx4 acc;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = acc0[i] + (acc1[i] + acc2[i]);
    return acc;
}

// MFMA network forward + input gradient for the T atoms of a tile (MFMA
// columns >= T are zero).  On entry G holds the BF16 (hi, lo) rows made by
// split_g_inplace; on return (GRAD) it holds dE/dG as fp32 [T][kLdG].
// fr points at the element's hi fragments; its lo fragments follow after
// FragLayout::Count fragments.
template <int T, bool SPLIT, bool GRAD>
__device__ __forceinline__ void mlp_mfma(const float* __restrict__ w, const bf16x8* __restrict__ fr, float* G,
                         MlpMfmaSmem<T, SPLIT>& sm, float* E, int tid, int nthr)
{
    using L = W32Layout;
    using F = FragLayout;
    constexpr int LO = SPLIT ? 1 : 0;
    const bf16x8* lo = fr + F::Count * 64;
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    const int col = lane & 15, rq = (lane >> 4) * 4;
    const bool live = col < T;
    const __bf16* ghi = reinterpret_cast<const __bf16*>(G);
    const __bf16* glo = ghi + T * kLdG;
    // layer 1: 160 x 384
    for (int mt = wave; mt < 10; mt += nw) {
        const int f = (F::F1 + mt * 12) * 64;
        const floatx4 acc = mfma_tile<T, 12, SPLIT>(fr + f, lo + f, ghi, glo, kLdG, lane);
        if (live) {
            const int o = mt * 16 + rq;
            const float4 b = *reinterpret_cast<const float4*>(w + L::B1 + o);
            const floatx4 z = {acc[0] + b.x, acc[1] + b.y, acc[2] + b.z, acc[3] + b.w};
            floatx4 h, d;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                h[i] = celu_f(z[i]);
                d[i] = celu_d(z[i]);
            }
            put_act4<SPLIT>(sm.h1[0], sm.h1[LO], col * kLd1 + o, h);
            *reinterpret_cast<floatx4*>(sm.d1 + col * kLdF1 + o) = d;
        }
    }
    __syncthreads();
    // layer 2: 128 x 160
    for (int mt = wave; mt < 8; mt += nw) {
        const int f = (F::F2 + mt * 5) * 64;
        const floatx4 acc = mfma_tile<T, 5, SPLIT>(fr + f, lo + f, sm.h1[0], sm.h1[LO], kLd1, lane);
        if (live) {
            const int o = mt * 16 + rq;
            const float4 b = *reinterpret_cast<const float4*>(w + L::B2 + o);
            const floatx4 z = {acc[0] + b.x, acc[1] + b.y, acc[2] + b.z, acc[3] + b.w};
            floatx4 h, d;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                h[i] = celu_f(z[i]);
                d[i] = celu_d(z[i]);
            }
            put_act4<SPLIT>(sm.h2[0], sm.h2[LO], col * kLd2 + o, h);
            *reinterpret_cast<floatx4*>(sm.d2 + col * kLdF2 + o) = d;
        }
    }
    __syncthreads();
    // layer 3: 96 x 128, fused with the output layer and delta3 = celu'(z3) W4
    for (int mt = wave; mt < 6; mt += nw) {
        const int f = (F::F3 + mt * 4) * 64;
        const floatx4 acc = mfma_tile<T, 4, SPLIT>(fr + f, lo + f, sm.h2[0], sm.h2[LO], kLd2, lane);
        float part = 0.f;
        const int o = mt * 16 + rq;
        const float4 b = *reinterpret_cast<const float4*>(w + L::B3 + o);
        const float4 w4 = *reinterpret_cast<const float4*>(w + L::W4 + o);
        const floatx4 z = {acc[0] + b.x, acc[1] + b.y, acc[2] + b.z, acc[3] + b.w};
        const floatx4 w4v = {w4.x, w4.y, w4.z, w4.w};
        floatx4 d3;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            part += w4v[i] * celu_f(z[i]);
            d3[i] = celu_d(z[i]) * w4v[i];
        }
        if (live) put_act4<SPLIT>(sm.h3[0], sm.h3[LO], col * kLd3 + o, d3);
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (lane < 16) sm.ep[mt * 16 + lane] = part;
    }
    __syncthreads();
    if (tid < T) {
        float s = w[L::B4];
        for (int mt = 0; mt < 6; ++mt) s += sm.ep[mt * 16 + tid];
        E[tid] = s;
    }
    if (!GRAD) return;
    // delta2 = celu'(z2) * W3^T delta3   (128 x 96)
    for (int mt = wave; mt < 8; mt += nw) {
        const int f = (F::B3 + mt * 3) * 64;
        const floatx4 acc = mfma_tile<T, 3, SPLIT>(fr + f, lo + f, sm.h3[0], sm.h3[LO], kLd3, lane);
        if (live) {
            const int o = mt * 16 + rq;
            const floatx4 d = *reinterpret_cast<const floatx4*>(sm.d2 + col * kLdF2 + o);
            const floatx4 v = {acc[0] * d[0], acc[1] * d[1], acc[2] * d[2], acc[3] * d[3]};
            put_act4<SPLIT>(sm.h2[0], sm.h2[LO], col * kLd2 + o, v);
        }
    }
    __syncthreads();
    // delta1 = celu'(z1) * W2^T delta2   (160 x 128)
    for (int mt = wave; mt < 10; mt += nw) {
        const int f = (F::B2 + mt * 4) * 64;
        const floatx4 acc = mfma_tile<T, 4, SPLIT>(fr + f, lo + f, sm.h2[0], sm.h2[LO], kLd2, lane);
        if (live) {
            const int o = mt * 16 + rq;
            const floatx4 d = *reinterpret_cast<const floatx4*>(sm.d1 + col * kLdF1 + o);
            const floatx4 v = {acc[0] * d[0], acc[1] * d[1], acc[2] * d[2], acc[3] * d[3]};
            put_act4<SPLIT>(sm.h1[0], sm.h1[LO], col * kLd1 + o, v);
        }
    }
    __syncthreads();
    // dE/dG = W1^T delta1   (384 x 160), written as fp32 over the (dead) G operand
    for (int mt = wave; mt < 24; mt += nw) {
        const int f = (F::B1 + mt * 5) * 64;
        const floatx4 acc = mfma_tile<T, 5, SPLIT>(fr + f, lo + f, sm.h1[0], sm.h1[LO], kLd1, lane);
        if (live) *reinterpret_cast<floatx4*>(G + col * kLdG + mt * 16 + rq) = acc;
    }
    __syncthreads();
}

// ------------------------------------------------------------------------
// FP8 (OCP E4M3, max 448) network: weights carry a static per-layer scale
// 448 / amax|W|; every B operand (descriptors, activations, deltas) is
// quantized per tile and layer with 448 / amax of that tile, so nothing
// saturates; FP32 accumulation, dequantised in the epilogue.
// ------------------------------------------------------------------------
constexpr int kLdQ = kNumFeat + 16;  // bytes per quantized row

template <int T>
struct MlpFp8Smem {
    float a1[T * kLdF1];         // h1, later delta1 (fp32)
    float a2[T * kLdF2];         // h2, later delta2
    float a3[T * kLdF3];         // delta3
    float d1[T * kLdF1];         // celu'(z1)
    float d2[T * kLdF2];         // celu'(z2)
    unsigned char q[T * kLdQ];   // quantized B operand of the current layer
    float ep[8 * 16];
    unsigned amax;
};

// src [T][ld] (first K columns) -> E4M3 rows of q scaled by 448 / amax;
// returns the inverse scale.  Workgroup-wide.
template <int T>
__device__ __forceinline__ float quantize_tile(const float* src, int ld, int K, unsigned char* q, unsigned* amax, int tid, int nthr)
{
    if (tid == 0) *amax = 0u;
    __syncthreads();
    float m = 0.f;
    for (int i = tid; i < T * K; i += nthr) m = fmaxf(m, fabsf(src[(i / K) * ld + i % K]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((tid & 63) == 0) atomicMax(amax, __float_as_uint(m));
    __syncthreads();
    const float am = __uint_as_float(*amax);
    const float sc = am > 0.f ? 448.f / am : 1.f;
    for (int i4 = tid; i4 < T * K / 4; i4 += nthr) {
        const int t = (4 * i4) / K, k = (4 * i4) % K;
        const float4 v = *reinterpret_cast<const float4*>(src + t * ld + k);
        int wd = __builtin_amdgcn_cvt_pk_fp8_f32(v.x * sc, v.y * sc, 0, false);
        wd = __builtin_amdgcn_cvt_pk_fp8_f32(v.z * sc, v.w * sc, wd, true);
        *reinterpret_cast<int*>(q + t * kLdQ + k) = wd;
    }
    __syncthreads();
    return 1.f / sc;
}

template <int T, int KT>
__device__ __forceinline__ floatx4 mfma_tile_fp8(const long* __restrict__ frag, const unsigned char* q, int lane)
{
    floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
    const int col = lane & 15, kq = (lane >> 4) * 8;
    const bool live = col < T;
    const unsigned char* row = q + (live ? col : 0) * kLdQ + kq;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
        const long a = frag[kt * 64 + lane];
        long b = *reinterpret_cast<const long*>(row + kt * 32);
        if (!live) b = 0;
        if (kt & 1)
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, acc1, 0, 0, 0);
        else
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, acc0, 0, 0, 0);
    }
    floatx4 acc;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = acc0[i] + acc1[i];
    return acc;
}

// FP8 network forward + input gradient.  G: fp32 [T][kLdG], replaced by
// dE/dG when GRAD.  ws: inverse weight scales of layers F1 F2 F3 B3 B2 B1.
template <int T, bool GRAD>
__device__ __forceinline__ void mlp_fp8(const float* __restrict__ w, const long* __restrict__ fr, const float* __restrict__ ws,
                        float* G, MlpFp8Smem<T>& sm, float* E, int tid, int nthr)
{
    using L = W32Layout;
    using F = FragLayout;
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    const int col = lane & 15, rq = (lane >> 4) * 4;
    const bool live = col < T;
    // layer 1: 160 x 384
    float dq = quantize_tile<T>(G, kLdG, kNumFeat, sm.q, &sm.amax, tid, nthr) * ws[0];
    for (int mt = wave; mt < 10; mt += nw) {
        const floatx4 acc = mfma_tile_fp8<T, 12>(fr + (F::F1 + mt * 12) * 64, sm.q, lane);
        if (live) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = mt * 16 + rq + i;
                const float z = acc[i] * dq + w[L::B1 + o];
                sm.a1[col * kLdF1 + o] = celu_f(z);
                sm.d1[col * kLdF1 + o] = celu_d(z);
            }
        }
    }
    __syncthreads();
    // layer 2: 128 x 160
    dq = quantize_tile<T>(sm.a1, kLdF1, kH1, sm.q, &sm.amax, tid, nthr) * ws[1];
    for (int mt = wave; mt < 8; mt += nw) {
        const floatx4 acc = mfma_tile_fp8<T, 5>(fr + (F::F2 + mt * 5) * 64, sm.q, lane);
        if (live) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = mt * 16 + rq + i;
                const float z = acc[i] * dq + w[L::B2 + o];
                sm.a2[col * kLdF2 + o] = celu_f(z);
                sm.d2[col * kLdF2 + o] = celu_d(z);
            }
        }
    }
    __syncthreads();
    // layer 3: 96 x 128 with the output layer and delta3 = celu'(z3) W4
    dq = quantize_tile<T>(sm.a2, kLdF2, kH2, sm.q, &sm.amax, tid, nthr) * ws[2];
    for (int mt = wave; mt < 6; mt += nw) {
        const floatx4 acc = mfma_tile_fp8<T, 4>(fr + (F::F3 + mt * 4) * 64, sm.q, lane);
        float part = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = mt * 16 + rq + i;
            const float z = acc[i] * dq + w[L::B3 + o];
            const float w4 = w[L::W4 + o];
            part += w4 * celu_f(z);
            if (live) sm.a3[col * kLdF3 + o] = celu_d(z) * w4;
        }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (lane < 16) sm.ep[mt * 16 + lane] = part;
    }
    __syncthreads();
    if (tid < T) {
        float s = w[L::B4];
        for (int mt = 0; mt < 6; ++mt) s += sm.ep[mt * 16 + tid];
        E[tid] = s;
    }
    if (!GRAD) return;
    // delta2 = celu'(z2) * W3^T delta3
    dq = quantize_tile<T>(sm.a3, kLdF3, kH3, sm.q, &sm.amax, tid, nthr) * ws[3];
    for (int mt = wave; mt < 8; mt += nw) {
        const floatx4 acc = mfma_tile_fp8<T, 3>(fr + (F::B3 + mt * 3) * 64, sm.q, lane);
        if (live) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = mt * 16 + rq + i;
                sm.a2[col * kLdF2 + o] = acc[i] * dq * sm.d2[col * kLdF2 + o];
            }
        }
    }
    __syncthreads();
    // delta1 = celu'(z1) * W2^T delta2
    dq = quantize_tile<T>(sm.a2, kLdF2, kH2, sm.q, &sm.amax, tid, nthr) * ws[4];
    for (int mt = wave; mt < 10; mt += nw) {
        const floatx4 acc = mfma_tile_fp8<T, 4>(fr + (F::B2 + mt * 4) * 64, sm.q, lane);
        if (live) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = mt * 16 + rq + i;
                sm.a1[col * kLdF1 + o] = acc[i] * dq * sm.d1[col * kLdF1 + o];
            }
        }
    }
    __syncthreads();
    // dE/dG = W1^T delta1
    dq = quantize_tile<T>(sm.a1, kLdF1, kH1, sm.q, &sm.amax, tid, nthr) * ws[5];
    for (int mt = wave; mt < 24; mt += nw) {
        const floatx4 acc = mfma_tile_fp8<T, 5>(fr + (F::B1 + mt * 5) * 64, sm.q, lane);
        if (live) {
#pragma unroll
            for (int i = 0; i < 4; ++i) G[col * kLdG + mt * 16 + rq + i] = acc[i] * dq;
        }
    }
    __syncthreads();
}

}  // namespace nnp
