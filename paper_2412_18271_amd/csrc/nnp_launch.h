// nnp_launch.h -- host-side launchers of the kernels in nnp_kernels.hip.
#pragma once

#include "nnp_internal.h"

namespace nnp {

// One energy (and, if grad, force) evaluation at the current positions.
// path 0 = plain (one kernel per stage), 1 = fused, 2 = split (descriptors,
// wide-tile network, adjoint: three kernels); mode 0 = FP32 VALU,
// 1 = BF16 MFMA, 2 = split BF16 MFMA (hi/lo operands, three products),
// 3 = E4M3 MFMA with per-layer scales.
// ev0 / ev1 (optional): events stamped by the first and the last kernel
// dispatch of the evaluation itself (start / end of execution).
hipError_t launch_eval(const Sys& S, int path, int mode, int T, bool grad, hipStream_t s,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Force sums -> FP64 + velocity Verlet + energies + step-state update (see
// kernel); ev0 / ev1 as for launch_eval.
hipError_t launch_gather_integrate(const Sys& S, double dt, int mode, hipStream_t s, bool forces = true,
                                   hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Stored-intermediates forward (pair list, descriptors -> S.G, network with
// dE/dG -> S.dG) and the adjoint from S.dG (plain-path kernels, tile size T).
hipError_t launch_store_forward(const Sys& S, int mode, int T, hipStream_t s);
hipError_t launch_adjoint(const Sys& S, hipStream_t s);
hipError_t launch_kickdrift(const Sys& S, double dt, hipStream_t s);
hipError_t launch_positions_in(const Sys& S, const void* src, int is_f64, hipStream_t s);
hipError_t launch_forces_out(const Sys& S, double* dst, hipStream_t s);
hipError_t launch_energy_out(const Sys& S, double* dst, hipStream_t s);
// Energies of the most recent evaluation -> energy log and Ecur / Kcur.
hipError_t launch_energy_flush(const Sys& S, hipStream_t s);
hipError_t launch_invalidate_lists(const Sys& S, hipStream_t s);
// Extra force providers: caller-order positions out and buffers cleared;
// then their forces and energies added to the running evaluation's sums.
hipError_t launch_extra_prepare(const Sys& S, double* pos, double* frc, double* en, hipStream_t s);
hipError_t launch_extra_add(const Sys& S, const double* frc, const double* en, hipStream_t s);
// E4M3 encoding of n floats by the device conversion instruction (format check).
hipError_t launch_fp8_encode(const float* x, int n, unsigned char* out, hipStream_t s);
hipError_t launch_descriptors_only(const Sys& S, hipStream_t s);
// Network of the split evaluation over S.wtiles (S.G -> S.Ei and, if grad,
// S.dG); mode 1 = BF16, 2 = split BF16; nblk = S.wide_blk.
hipError_t launch_mlp_wide(const Sys& S, int mode, int nblk, bool grad, hipStream_t s, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr);

}  // namespace nnp
