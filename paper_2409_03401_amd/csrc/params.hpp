// Kernel parameter block and storage formats shared by the kernels and the host API.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

// D3Q19 fluid + 3 x D3Q19 scalars (the paper's lattices), or D3Q19 + 4 x D3Q7 (a third
// composition on the reduced lattice)
constexpr int kMaxSlots = 19 + 3 * 19;
// moments written by the moments mode: phi, cA, cB, muA, muB, p, ux, uy, uz, then cC, muC
// of a third composition (N components)
constexpr int kNumMom = 11;
constexpr int kNumDiag = 8;

enum Prec : int { P64 = 0, P32 = 1, P16 = 2, PB16 = 3 };
// MODE_STEP_PHI: a step that also writes phi of its source state (P.phi_out)
enum Mode : int { MODE_STEP = 0, MODE_MOMENTS = 1, MODE_DIAG = 2, MODE_STEP_PHI = 3 };
// collision operator of the fused step: the paper's BGK, or two relaxation times
// (flags): COLL_TRT two relaxation times, COLL_VD the variable-density flow model
// COLL_GK general curvature matrices of the free energies (2 x 2 closure per node)
// COLL_MRT multiple relaxation times on the lattice's moment basis
enum Coll : int { COLL_BGK = 0, COLL_TRT = 1, COLL_VD = 2, COLL_GK = 4, COLL_MRT = 8 };

// Storage traits.  FP64 / FP32 store every population as is.  The 16-bit
// formats store the moving populations (k != 0) as d = (x - w_k ref) * 2^s in
// FP16 / BF16 (round to nearest even) and keep the rest population (k = 0) in
// FP32: the rest populations carry most of the conserved composition, so their
// rounding would otherwise break mass conservation at the 16-bit level.
template <int PREC> struct Stor;
template <> struct Stor<P64> { using T = double; using R = double; using C = double; };
template <> struct Stor<P32> { using T = float; using R = float; using C = float; };
template <> struct Stor<P16> { using T = __half; using R = float; using C = float; };
template <> struct Stor<PB16> { using T = __hip_bfloat16; using R = float; using C = float; };

__host__ __device__ inline constexpr int slot_bytes(int prec, int k) {
    return prec == P64 ? 8 : (prec == P32 ? 4 : (k == 0 ? 4 : 2));
}

struct KParams {
    // grid (kernel frame: 2D problems live in the x-z plane with ny = 1)
    int nx, ny, nz;
    int wall_x, wall_y, wall_z;  // 1: half-way bounce-back walls on that axis
    int zc;                      // planes marched per work-group
    int tiles_x, tiles_y, tiles_z;  // work-group tiles per axis (tiles_z = z chunks)
    int mean_subtract;           // buoyancy uses phi - phi_ref
    // model (Section 2), lattice units
    double W, lam, mphi_w2;      // mphi_w2 = M_phi / W^2 = 1 / tau_phi
    double c0A, c0B, c1A, c1B;   // equilibrium compositions of phases 0 and 1
    double omega_g;              // g-lattice rate 1 / (M_phi / c_s^2 + 1/2)
    // TRT (COLL_TRT): magic parameters of f and of the scalar lattices; symmetric rate of g
    double trt_lf, trt_ls, omega_gp;
    int variable_density;        // 1: f holds dimensionless populations (rho(phi) model)
    // MRT (COLL_MRT): free rates of f (bulk, third, fourth order) and of g, h (second,
    // third, fourth order)
    double mrt_f[3], mrt_s[3];
    // general curvatures: kappa_pi = (k_AA, k_AB, k_BB) of phases 0 and 1 (dc/dmu of each
    // phase); general_k = 0 is the paper's identity
    double kap0[3], kap1[3];
    int general_k;
    double MA0, MA1, MB0, MB1;   // species mobilities per phase
    // a third independent composition C (N components; the kernels instantiated with
    // three compositions use it): equilibrium compositions and mobilities per phase
    double c0C, c1C, MC0, MC1;
    double nu0, nu1, rho0, drho;
    double gx, gy, gz;           // gravity in the kernel frame
    double cap;                  // 3/2 sigma W of Eq. SurfaceTension_Force
    double inv_W2;
    double dK_dW, dcap_dW;       // -2 M_phi / W^3 and 3/2 sigma (adjoint: d/dW)
    // FP32 copies of the constants the FP32 collision uses (one SGPR each, no
    // conversion in the loop)
    struct {
        float cap, inv_W2, drho, gx, gy, gz, inv_rho0, rho0, nu0, nu1, omega_g, MA0, MA1, MB0, MB1, MC0, MC1;
        float trt_lf, trt_ls, omega_gp;
        float mrt_f[3], mrt_s[3];
    } f32;
    // population copies addressed by the fused kernel: slot s of a copy starts at
    // base + (#moving slots before s) * stride_m + (#rest slots before s) * stride_r
    const char* src_base;
    char* dst_base;
    unsigned long long stride_m, stride_r;
    // 16-bit storage per field (0 f, 1 g, 2 hA, 3 hB, 4 hC): moving population k is
    // value = w_k fref + d * finv, d = (value - w_k fref) * fscale
    float fref[5], fscale[5], finv[5];
    // device scalars
    const double* phi_ref;       // buoyancy reference <phi> (aux area)
    double* partials;            // per-work-group partial sums
    // moments output (MODE_MOMENTS): phi, cA, cB, muA, muB, p, ux, uy, uz (kernel frame),
    // then cC, muC of a third composition
    void* mout[kNumMom];
    int mout_f32;
    // MODE_DIAG: 1 where phi >= 1/2, else 0, one byte per node (kernel frame)
    unsigned char* mask_out;
    // initialisation: given compositions c^A, c^B (, c^C) ([node]) instead of the closure,
    // or null
    const double* init_c[3];
    // adjoint kernels.  The adjoint of the arriving
    // population X_s(x) is lambda_s(x) plus, for a scalar population of field F
    // (g, h^A, h^B), the field-wide term c_F(x) (row F - 1 of auxc).  lambda is FP32
    // [slot][node] with slot stride adj_stride bytes.  aux holds the per-step FP32
    // [row][node] scratch: rows 0-2 dL/dG, 3 dL/dN, 4 dphi/dphi*, 5 q of dphi/dc,
    // 6 dphi/dK; auxc the three c_F rows (part of the adjoint state), same row stride.
    const char* adj_in;
    char* adj_out;
    unsigned long long adj_stride;
    float* aux;
    float* auxc;
    unsigned long long aux_stride;  // elements per aux row
    // MODE_STEP: when set, receives *phi_ref (steps between caller checkpoints)
    double* ref_copy;
    // MODE_STEP_PHI: receives phi of the source state ([node], compute type)
    void* phi_out;
    // absolute base of every slot of the source and the destination copy (canonical slot
    // order; filled on the host from src_base / dst_base).  The fused kernel reads them
    // from the kernel-argument segment (this block is its only argument, at offset 0)
    // with one scalar load per slot and plane instead of 64-bit scalar arithmetic.
    const char* src_slot[kMaxSlots];
    char* dst_slot[kMaxSlots];
};

constexpr int kAuxRows = 7;  // per-step scratch rows of the adjoint (c_F rows apart)
constexpr int kAuxCRows = 3;

// Euler characteristic of the closed cells of a node mask (droplet count of
// Section 4.2.2).  Only the d active axes of the run are listed: axis i has n[i]
// cells, mask stride stride[i], wall[i] != 0 when it ends at walls.  An anchor
// j_i in [0, n[i] + wall[i]) stands for the vertex position between cells j_i - 1
// and j_i and for cell j_i (when j_i < n[i]); nanchors = prod(n[i] + wall[i]).
struct EulerGeom {
    int d;
    int n[3], wall[3];
    long long stride[3];
    long long nanchors;
};

}  // namespace lbm
