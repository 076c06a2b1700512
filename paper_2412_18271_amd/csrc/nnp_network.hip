// nnp_network.hip -- the per-element network over wide tiles of atoms (the
// split evaluation: descriptors -> G in HBM, this kernel -> dE/dG in HBM,
// then the adjoint).
//
// A workgroup takes up to 16 NBLK consecutive atoms of one element (atoms are
// element-major in the internal order, so a wide tile is a contiguous range)
// and runs the network forward and its input gradient as six GEMMs on the
// MFMA units.  Each weight fragment read from L2 serves NBLK 16-atom column
// blocks, against one in the fused kernels: with NBLK = 4 the weight bytes
// per atom are a quarter of those of a 16-atom tile and 4/10 of a 10-atom
// tile.
//
// Wave w of the 8 computes output row tiles w, w + 8, ... of each layer for
// all NBLK column blocks: the A operands (pre-swizzled weight fragments,
// 16 rows x 32 k, the layout of the fused kernels) are read once per
// workgroup, the B operands (activations, BF16 hi and, split, lo rows) come
// from LDS.  Activations are written once by the producing layer's epilogue.
// In the split mode celu'(z) is recovered from h = celu(z) (hi + lo) as
// 1 for h > 0 and 1 + h / alpha otherwise (exp(z / alpha) = 1 + h / alpha),
// so the backward overwrites h in place and no FP32 derivative rows are
// kept; the single-pass mode keeps celu'(z) in FP32 rows, as the fused
// kernels do.
#include "nnp_device.h"
#include <hip/hip_ext.h>

#include "nnp_launch.h"

namespace nnp {

namespace {

constexpr int kWideThreads = 512;
constexpr int kWideWaves = kWideThreads / 64;

template <int NBLK, bool SPLIT>
struct WideSmem {
    static constexpr int NA = 16 * NBLK;
    static constexpr int NL = SPLIT ? 2 : 1;
    union {
        __bf16 g[NL * NA * kLdG];  // layer-1 operand: hi rows, then lo rows
        struct {
            __bf16 h2[NL * NA * kLd2];  // h2, then delta2
            __bf16 h3[NL * NA * kLd3];  // delta3
        } b;
    } u;
    __bf16 h1[NL * NA * kLd1];  // h1, then delta1
    float d1[SPLIT ? 1 : NA * kLdF1];
    float d2[SPLIT ? 1 : NA * kLdF2];
    float ep[6 * NA];  // output-layer partial sums per (row tile, atom)
};

// acc[nb] = rows 16 mt.. of W (fragments fhi / flo, KT k steps) times the
// B rows of column block nb (LDS, stride ld; lo rows at blo).  The k loop is
// unrolled completely and the A fragments of the next 2-3 steps are
// requested before the MFMAs of the current one: with two waves per SIMD
// the L2 latency of a fragment is otherwise exposed at every step.

template <int NBLK, int KT, bool SPLIT>
__device__ __forceinline__ void wide_gemm(const bf16x8* __restrict__ fhi, const bf16x8* __restrict__ flo,
                                          const __bf16* bhi, const __bf16* blo, int ld, int lane,
                                          floatx4 (&acc)[NBLK])
{
    // two accumulators per column block (hi*hi; the two lo products), or,
    // single-pass with one block, even and odd k steps: independent MFMA
    // chains
    floatx4 a0[NBLK], a1[NBLK];
#pragma unroll
    for (int nb = 0; nb < NBLK; ++nb) a0[nb] = a1[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int off = (lane & 15) * ld + (lane >> 4) * 8;
    constexpr int kPrefetch = SPLIT && NBLK == 2 ? 2 : 3;  // two workgroups per CU: 128 registers
    constexpr int R = kPrefetch + 1;
    bf16x8 ah[R], al[R];
#pragma unroll
    for (int k = 0; k < kPrefetch && k < KT; ++k) {
        ah[k] = fhi[k * 64 + lane];
        if constexpr (SPLIT) al[k] = flo[k * 64 + lane];
    }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
        if (kt + kPrefetch < KT) {
            ah[(kt + kPrefetch) % R] = fhi[(kt + kPrefetch) * 64 + lane];
            if constexpr (SPLIT) al[(kt + kPrefetch) % R] = flo[(kt + kPrefetch) * 64 + lane];
        }
        const bf16x8 h = ah[kt % R];
#pragma unroll
        for (int nb = 0; nb < NBLK; ++nb) {
            const int o = off + nb * 16 * ld + kt * 32;
            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(bhi + o);
            if constexpr (SPLIT) {
                const bf16x8 bl = *reinterpret_cast<const bf16x8*>(blo + o);
                a0[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bh, a0[nb], 0, 0, 0);
                a1[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bl, a1[nb], 0, 0, 0);
                a1[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[kt % R], bh, a1[nb], 0, 0, 0);
            } else if (NBLK == 1 && (kt & 1)) {
                a1[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bh, a1[nb], 0, 0, 0);
            } else {
                a0[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bh, a0[nb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int nb = 0; nb < NBLK; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[nb][i] = a0[nb][i] + a1[nb][i];
}

// Four consecutive activations of row `col` at column idx of a buffer with
// hi rows at p and lo rows NA * ld further.
template <bool SPLIT>
__device__ __forceinline__ floatx4 get_act4(const __bf16* p, int lo_off, int idx)
{
    const bf16x4 h = *reinterpret_cast<const bf16x4*>(p + idx);
    floatx4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = (float)h[i];
    if constexpr (SPLIT) {
        const bf16x4 l = *reinterpret_cast<const bf16x4*>(p + lo_off + idx);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] += (float)l[i];
    }
    return v;
}

__device__ __forceinline__ float celu_d_from_h(float h) { return h > 0.0f ? 1.0f : 1.0f + h * (1.0f / kCeluAlpha); }

}  // namespace

template <int NBLK, bool SPLIT, bool GRAD>
__global__ __launch_bounds__(kWideThreads) __attribute__((amdgpu_waves_per_eu(NBLK <= 2 ? 4 : 2))) void k_mlp_wide(Sys S)
{
    using F = FragLayout;
    using L = W32Layout;
    using Smem = WideSmem<NBLK, SPLIT>;
    constexpr int NA = Smem::NA;
    constexpr int LO = SPLIT ? 1 : 0;  // lo rows follow the hi rows (else alias them)
    __shared__ __attribute__((aligned(16))) Smem sm;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int4 t = S.wtiles[blockIdx.x];
    const int first = t.x, cnt = t.y, elem = t.z;
    const float* __restrict__ w = S.w32 + (size_t)elem * L::Stride;
    const bf16x8* __restrict__ fr = reinterpret_cast<const bf16x8*>(S.wfrag) + (size_t)elem * 2 * F::Count * 64;
    const bf16x8* __restrict__ frl = fr + F::Count * 64;
    const int col = lane & 15, rq = (lane >> 4) * 4;

    // G rows of the tile's atoms -> BF16 hi (and lo) rows; missing atoms
    // zero.  Every load is issued before the first conversion.
    {
        constexpr int PER = NA * (kNumFeat / 4) / kWideThreads;
        static_assert(PER * kWideThreads == NA * (kNumFeat / 4), "whole float4 rows per thread");
        float4 v[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = tid + q * kWideThreads, c = i / (kNumFeat / 4), f = (i - c * (kNumFeat / 4)) * 4;
            v[q] = c < cnt ? *reinterpret_cast<const float4*>(S.G + (size_t)(first + c) * kNumFeat + f)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = tid + q * kWideThreads, c = i / (kNumFeat / 4), f = (i - c * (kNumFeat / 4)) * 4;
            put_act4<SPLIT>(sm.u.g, sm.u.g + LO * NA * kLdG, c * kLdG + f, floatx4{v[q].x, v[q].y, v[q].z, v[q].w});
        }
    }
    __syncthreads();
    // layer 1: h1 = celu(W1 G + b1)   (160 x 384)
    for (int mt = wave; mt < 10; mt += kWideWaves) {
        const int f = (F::F1 + mt * 12) * 64;
        floatx4 acc[NBLK];
        wide_gemm<NBLK, 12, SPLIT>(fr + f, frl + f, sm.u.g, sm.u.g + LO * NA * kLdG, kLdG, lane, acc);
        const int o = mt * 16 + rq;
        const float4 b = *reinterpret_cast<const float4*>(w + L::B1 + o);
#pragma unroll
        for (int nb = 0; nb < NBLK; ++nb) {
            const int c = nb * 16 + col;
            const floatx4 z = {acc[nb][0] + b.x, acc[nb][1] + b.y, acc[nb][2] + b.z, acc[nb][3] + b.w};
            floatx4 h, d;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                h[i] = celu_f(z[i]);
                d[i] = celu_d(z[i]);
            }
            put_act4<SPLIT>(sm.h1, sm.h1 + LO * NA * kLd1, c * kLd1 + o, h);
            if constexpr (!SPLIT) *reinterpret_cast<floatx4*>(sm.d1 + c * kLdF1 + o) = d;
        }
    }
    __syncthreads();
    // layer 2: h2 = celu(W2 h1 + b2)   (128 x 160); h2 overlays G
    for (int mt = wave; mt < 8; mt += kWideWaves) {
        const int f = (F::F2 + mt * 5) * 64;
        floatx4 acc[NBLK];
        wide_gemm<NBLK, 5, SPLIT>(fr + f, frl + f, sm.h1, sm.h1 + LO * NA * kLd1, kLd1, lane, acc);
        const int o = mt * 16 + rq;
        const float4 b = *reinterpret_cast<const float4*>(w + L::B2 + o);
#pragma unroll
        for (int nb = 0; nb < NBLK; ++nb) {
            const int c = nb * 16 + col;
            const floatx4 z = {acc[nb][0] + b.x, acc[nb][1] + b.y, acc[nb][2] + b.z, acc[nb][3] + b.w};
            floatx4 h, d;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                h[i] = celu_f(z[i]);
                d[i] = celu_d(z[i]);
            }
            put_act4<SPLIT>(sm.u.b.h2, sm.u.b.h2 + LO * NA * kLd2, c * kLd2 + o, h);
            if constexpr (!SPLIT) *reinterpret_cast<floatx4*>(sm.d2 + c * kLdF2 + o) = d;
        }
    }
    __syncthreads();
    // layer 3 (96 x 128) with the output layer: E partial sums and
    // delta3 = celu'(z3) W4
    for (int mt = wave; mt < 6; mt += kWideWaves) {
        const int f = (F::F3 + mt * 4) * 64;
        floatx4 acc[NBLK];
        wide_gemm<NBLK, 4, SPLIT>(fr + f, frl + f, sm.u.b.h2, sm.u.b.h2 + LO * NA * kLd2, kLd2, lane, acc);
        const int o = mt * 16 + rq;
        const float4 b = *reinterpret_cast<const float4*>(w + L::B3 + o);
        const float4 w4 = *reinterpret_cast<const float4*>(w + L::W4 + o);
        const floatx4 w4v = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
        for (int nb = 0; nb < NBLK; ++nb) {
            const int c = nb * 16 + col;
            const floatx4 z = {acc[nb][0] + b.x, acc[nb][1] + b.y, acc[nb][2] + b.z, acc[nb][3] + b.w};
            float part = 0.f;
            floatx4 d3;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                part += w4v[i] * celu_f(z[i]);
                d3[i] = celu_d(z[i]) * w4v[i];
            }
            put_act4<SPLIT>(sm.u.b.h3, sm.u.b.h3 + LO * NA * kLd3, c * kLd3 + o, d3);
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            if (lane < 16) sm.ep[mt * NA + c] = part;
        }
    }
    __syncthreads();
    for (int c = tid; c < cnt; c += kWideThreads) {
        float e = w[L::B4];
        for (int mt = 0; mt < 6; ++mt) e += sm.ep[mt * NA + c];
        S.Ei[first + c] = e;
    }
    if constexpr (GRAD) {
        // delta2 = celu'(z2) * W3^T delta3   (128 x 96), over h2 in place
        for (int mt = wave; mt < 8; mt += kWideWaves) {
            const int f = (F::B3 + mt * 3) * 64;
            floatx4 acc[NBLK];
            wide_gemm<NBLK, 3, SPLIT>(fr + f, frl + f, sm.u.b.h3, sm.u.b.h3 + LO * NA * kLd3, kLd3, lane, acc);
            const int o = mt * 16 + rq;
#pragma unroll
            for (int nb = 0; nb < NBLK; ++nb) {
                const int c = nb * 16 + col;
                floatx4 d;
                if constexpr (SPLIT) {
                    const floatx4 h = get_act4<true>(sm.u.b.h2, NA * kLd2, c * kLd2 + o);
#pragma unroll
                    for (int i = 0; i < 4; ++i) d[i] = celu_d_from_h(h[i]);
                } else {
                    d = *reinterpret_cast<const floatx4*>(sm.d2 + c * kLdF2 + o);
                }
                const floatx4 v = {acc[nb][0] * d[0], acc[nb][1] * d[1], acc[nb][2] * d[2], acc[nb][3] * d[3]};
                put_act4<SPLIT>(sm.u.b.h2, sm.u.b.h2 + LO * NA * kLd2, c * kLd2 + o, v);
            }
        }
        __syncthreads();
        // delta1 = celu'(z1) * W2^T delta2   (160 x 128), over h1 in place
        for (int mt = wave; mt < 10; mt += kWideWaves) {
            const int f = (F::B2 + mt * 4) * 64;
            floatx4 acc[NBLK];
            wide_gemm<NBLK, 4, SPLIT>(fr + f, frl + f, sm.u.b.h2, sm.u.b.h2 + LO * NA * kLd2, kLd2, lane, acc);
            const int o = mt * 16 + rq;
#pragma unroll
            for (int nb = 0; nb < NBLK; ++nb) {
                const int c = nb * 16 + col;
                floatx4 d;
                if constexpr (SPLIT) {
                    const floatx4 h = get_act4<true>(sm.h1, NA * kLd1, c * kLd1 + o);
#pragma unroll
                    for (int i = 0; i < 4; ++i) d[i] = celu_d_from_h(h[i]);
                } else {
                    d = *reinterpret_cast<const floatx4*>(sm.d1 + c * kLdF1 + o);
                }
                const floatx4 v = {acc[nb][0] * d[0], acc[nb][1] * d[1], acc[nb][2] * d[2], acc[nb][3] * d[3]};
                put_act4<SPLIT>(sm.h1, sm.h1 + LO * NA * kLd1, c * kLd1 + o, v);
            }
        }
        __syncthreads();
        // dE/dG = W1^T delta1   (384 x 160) -> HBM
        for (int mt = wave; mt < 24; mt += kWideWaves) {
            const int f = (F::B1 + mt * 5) * 64;
            floatx4 acc[NBLK];
            wide_gemm<NBLK, 5, SPLIT>(fr + f, frl + f, sm.h1, sm.h1 + LO * NA * kLd1, kLd1, lane, acc);
            const int o = mt * 16 + rq;
#pragma unroll
            for (int nb = 0; nb < NBLK; ++nb) {
                const int c = nb * 16 + col;
                if (c < cnt)
                    *reinterpret_cast<float4*>(S.dG + (size_t)(first + c) * kNumFeat + o) =
                        make_float4(acc[nb][0], acc[nb][1], acc[nb][2], acc[nb][3]);
            }
        }
    }
}

template <int NBLK, bool SPLIT>
static hipError_t launch_wide_t(const Sys& S, bool grad, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (grad)
        hipExtLaunchKernelGGL((k_mlp_wide<NBLK, SPLIT, true>), dim3(S.nwtiles), dim3(kWideThreads), 0, s, ev0, ev1,
                              0, S);
    else
        hipExtLaunchKernelGGL((k_mlp_wide<NBLK, SPLIT, false>), dim3(S.nwtiles), dim3(kWideThreads), 0, s, ev0, ev1,
                              0, S);
    return hipGetLastError();
}

hipError_t launch_mlp_wide(const Sys& S, int mode, int nblk, bool grad, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (S.nwtiles <= 0) return hipSuccess;
#define NNP_WIDE(NB)                                                                  \
    if (nblk == NB) {                                                                 \
        if (mode == 2) return launch_wide_t<NB, true>(S, grad, s, ev0, ev1);          \
        if (mode == 1) return launch_wide_t<NB, false>(S, grad, s, ev0, ev1);         \
    }
    NNP_WIDE(1)
    NNP_WIDE(2)
    NNP_WIDE(3)
    NNP_WIDE(4)
#undef NNP_WIDE
    return hipErrorInvalidValue;
}

}  // namespace nnp
