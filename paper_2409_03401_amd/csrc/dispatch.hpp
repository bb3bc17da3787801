// Launchers of one lattice family at one storage precision, used by the host API.
#pragma once

#include "params.hpp"

namespace lbm {

struct KernelSet {
    // fused kernel in MODE_STEP / MODE_MOMENTS / MODE_DIAG
    void (*fused)(int mode, dim3 grid, const KParams& kp, hipStream_t s);
    // equilibrium initialisation, one thread per node (muC0: the third composition's
    // potential, families with three compositions only)
    void (*init)(const KParams& kp, const double* phi0, const double* muA0, const double* muB0,
                 const double* muC0, hipStream_t s);
    void (*get_pops)(const KParams& kp, int nslots, long long nodes, double* out, hipStream_t s);
    void (*set_pops)(const KParams& kp, int nslots, long long nodes, const double* in, hipStream_t s);
    // bounce-back fix-up on the two faces of one wall axis (0 x, 1 y), after a step (z
    // walls bounce back when the next step pulls)
    void (*walls)(const KParams& kp, int axis, hipStream_t s);
    // adjoint: nullptr when the storage precision has no adjoint (16-bit formats)
    void (*adj_step)(const KParams& kp, long long nodes, const void* phi, hipStream_t s);
    void (*adj_seed)(const KParams& kp, long long nodes, const double* dL_dphi, hipStream_t s);
    void (*adj_gather)(const KParams& kp, long long nodes, int mode, double* grad_phi0, hipStream_t s);
    void (*adj_init_local)(const KParams& kp, long long nodes, const double* phi0, const double* muA0,
                           const double* muB0, hipStream_t s);
    // adjoint to (set = false) or from (set = true) an FP64 [slot][node] array
    void (*adj_copy)(const KParams& kp, int nslots, long long nodes, double* buf, bool set, hipStream_t s);
    int tx, ty;  // work-group tile of the fused kernel
};

// fluid: 0 (none) or 9 / 19; prec: Prec; (tx, ty): work-group tile, 0 for the
// default.  nullptr for unsupported combinations.
const KernelSet* kernels_2d(int fluid, int prec, int tx);
const KernelSet* kernels_3d(int fluid, int prec, int tx, int ty);
// the paper's scalar lattices (D2Q9 / D3Q19 for g, h^A, h^B): all precisions, adjoint at FP64 / FP32
const KernelSet* kernels_paper_2d(int fluid, int prec);
const KernelSet* kernels_paper_3d(int fluid, int prec);
// the two-relaxation-time collision (scalar lattice 5 / 9 in 2D, 7 / 19 in 3D): all precisions, no adjoint
const KernelSet* kernels_trt_2d(int scalar, int fluid, int prec);
const KernelSet* kernels_trt_3d(int scalar, int fluid, int prec);
// the multiple-relaxation-time collision (same lattice pairs): all precisions, no adjoint
const KernelSet* kernels_mrt_2d(int scalar, int fluid, int prec);
const KernelSet* kernels_mrt_3d(int scalar, int fluid, int prec);
// the variable-density flow model (needs the fluid lattice): all precisions, no adjoint
const KernelSet* kernels_vd_2d(int scalar, bool trt, int prec);
const KernelSet* kernels_vd_3d(int scalar, bool trt, int prec);
// general curvature matrices of the free energies (BGK, Boussinesq): all precisions, no adjoint
const KernelSet* kernels_gk_2d(int scalar, int fluid, int prec);
const KernelSet* kernels_gk_3d(int scalar, int fluid, int prec);
// a third independent composition (N components) on the reduced scalar lattices (D2Q5 /
// D3Q7), BGK Boussinesq step: all precisions, no adjoint
const KernelSet* kernels_nc3_2d(int fluid, int prec);
const KernelSet* kernels_nc3_3d(int fluid, int prec);

void launch_sum_partials(const double* v, long long n, double* partials, int nblocks, hipStream_t s);
// width 1, 8, or 9 (the diagnostics with a third composition: entry 8 goes to out[10])
void launch_finalize(const double* partials, int nparts, int width, int maxslot, double scale0,
                     double* out, hipStream_t s);
// out[0..5] (+)= sum of [nparts][6] partials (parameter gradients)
void launch_sum6(const double* partials, int nparts, double* out, bool accumulate, hipStream_t s);
void launch_zero(double* p, long long n, hipStream_t s);
// Euler characteristic of a node mask: partials[0 .. nblocks) receive the sums of
// nblocks work-groups striding over the anchors
void launch_euler(const unsigned char* mask, const EulerGeom& g, double* partials, int nblocks, hipStream_t s);

}  // namespace lbm
