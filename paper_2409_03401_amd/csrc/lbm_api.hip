// C ABI of the library (declared in include/lbm.h): configuration checks, state
// layout, launch geometry and the host side of every entry point.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "dispatch.hpp"
#include "lattice.hpp"
#include "lbm.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define LBM_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) return fail(LBM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
// aux area: kAuxHead doubles of scalars (0: buoyancy reference <phi>, 8..: the
// diagnostics), then the per-work-group partial sums
constexpr int kAuxHead = 32;
size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    const KernelSet* ks;
    int dim, qf, qs, nslots, prec;
    int nc;  // independent compositions (2: the ternary fluid, 3: A, B, C)
    int NX, NY, NZ;  // kernel frame
    long long nodes;
    size_t slot_off[kMaxSlots];
    size_t copy_bytes;
    size_t stride_m, stride_r;  // bytes of a moving / rest slot
    int tx, ty, zc;
    int tiles[3];
    dim3 grid;        // 1D: one work-group per tile
    long long nparts;     // work-groups of the fused kernel
    size_t aux_bytes;
    size_t mask_off;  // diagnostics mask (1 byte per node) after the aux area
    size_t state_bytes;
    // adjoint workspace: the adjoint state (two FP32 lambda copies, kAuxCRows FP32 rows of
    // c_F), then the per-step scratch (kAuxRows FP32 rows, theta partials of the adjoint
    // kernels (6 per 256-node work-group), phi of a state)
    size_t adj_stride, aux_stride_elems, adj_bytes;
    size_t adj_state_bytes, adj_scratch_bytes;  // the two parts of adj_bytes
    long long adj_parts;
};

int check_config(const lbm_config* c, Layout* L) {
    if (!c) return fail(LBM_EINVAL, "config is NULL");
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(LBM_EINVAL, "grid sizes must be >= 1");
    if (c->dim != 0 && c->dim != 2 && c->dim != 3) return fail(LBM_EINVAL, "dim must be 0, 2 or 3");
    if (c->scalar == LBM_D2Q5 || c->scalar == LBM_D2Q9) {
        if (c->nz != 1) return fail(LBM_EINVAL, "2D scalar lattices need nz = 1");
        if (c->fluid != LBM_NONE && c->fluid != LBM_D2Q9)
            return fail(LBM_EUNSUPPORTED, "2D runs take LBM_NONE or LBM_D2Q9 for the fluid");
        L->dim = 2;
    } else if (c->scalar == LBM_D3Q7 || c->scalar == LBM_D3Q19) {
        if (c->fluid != LBM_NONE && c->fluid != LBM_D3Q19)
            return fail(LBM_EUNSUPPORTED, "3D runs take LBM_NONE or LBM_D3Q19 for the fluid");
        L->dim = 3;
    } else {
        return fail(LBM_EUNSUPPORTED, "scalar lattice must be LBM_D2Q5, LBM_D2Q9, LBM_D3Q7 or LBM_D3Q19");
    }
    if (c->dim != 0 && c->dim != L->dim) return fail(LBM_EINVAL, "dim does not match the scalar lattice");
    const bool paper_scalar = c->scalar == LBM_D2Q9 || c->scalar == LBM_D3Q19;
    if (c->collision != LBM_BGK && c->collision != LBM_TRT && c->collision != LBM_MRT)
        return fail(LBM_EINVAL, "collision must be LBM_BGK, LBM_TRT or LBM_MRT");
    const bool trt = c->collision == LBM_TRT;
    const bool mrt = c->collision == LBM_MRT;
    if (mrt)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j)
                if (!(c->mrt_rates[i][j] > 0 && c->mrt_rates[i][j] < 2))
                    return fail(LBM_EUNSTABLE, "mrt_rates must lie in (0, 2)");
    if (c->variable_density != 0 && c->variable_density != 1)
        return fail(LBM_EINVAL, "variable_density must be 0 or 1");
    const bool vd = c->variable_density == 1;
    if (c->general_kappa != 0 && c->general_kappa != 1) return fail(LBM_EINVAL, "general_kappa must be 0 or 1");
    const bool gk = c->general_kappa == 1;
    if (gk) {
        for (int pi = 0; pi < 2; ++pi) {
            const double* k = c->kappa[pi];
            if (!(std::isfinite(k[0]) && std::isfinite(k[1]) && std::isfinite(k[2])))
                return fail(LBM_EINVAL, "kappa must be finite");
            if (!(k[0] > 0 && k[0] * k[2] - k[1] * k[1] > 0))
                return fail(LBM_EINVAL, "kappa must be symmetric positive definite");
            // the reduced composition lattices grow a checkerboard mode once
            // (1 - w_0) exceeds the smallest eigenvalue of kappa (D2Q5: 2/3, D3Q7: 3/4)
            const double lmin = 0.5 * (k[0] + k[2]) - std::sqrt(0.25 * (k[0] - k[2]) * (k[0] - k[2]) + k[1] * k[1]);
            const double one_minus_w0 = c->scalar == LBM_D2Q5 ? 2.0 / 3.0 : c->scalar == LBM_D3Q7 ? 0.75 : 0.0;
            if (lmin < one_minus_w0)
                return fail(LBM_EUNSTABLE, "kappa's smallest eigenvalue is below 1 - w_0 of the D2Q5 / D3Q7 lattice");
        }
        if (trt || mrt || vd) return fail(LBM_EUNSUPPORTED, "general_kappa runs with the BGK Boussinesq step");
    }
    if (vd && c->fluid == LBM_NONE) return fail(LBM_EINVAL, "variable_density needs a fluid lattice");
    if (vd && !(c->rho0 + c->drho > 0)) return fail(LBM_EINVAL, "variable_density needs rho0 + drho > 0");
    if (trt)
        for (double m : {c->trt_magic[0], c->trt_magic[1]})
            if (!(std::isfinite(m) && m > 0)) return fail(LBM_EINVAL, "trt_magic must be finite and > 0");
    if (c->precision < LBM_FP64 || c->precision > LBM_FP32_BF16STORE)
        return fail(LBM_EUNSUPPORTED, "unknown precision");
    for (int a = 0; a < 3; ++a)
        if (c->bc[a] != LBM_PERIODIC && c->bc[a] != LBM_WALLS)
            return fail(LBM_EINVAL, "bc must be LBM_PERIODIC or LBM_WALLS");
    const long long nodes = (long long)c->nx * c->ny * c->nz;
    if (nodes >= (1LL << 31)) return fail(LBM_EUNSUPPORTED, "more than 2^31 - 1 nodes");
    // kernels address a slot with a 32-bit byte offset: nodes x (8 B FP64, else 4 B) < 2^32
    if ((unsigned long long)nodes * (c->precision == LBM_FP64 ? 8ull : 4ull) > 0xFFFFFFFFull)
        return fail(LBM_EUNSUPPORTED, "grid too large for 32-bit slot offsets (FP64: < 2^29 nodes, else < 2^30)");
    const bool flow = c->fluid != LBM_NONE;
    if (c->gravity_mean_subtract && !flow)
        return fail(LBM_EINVAL, "gravity_mean_subtract needs a fluid lattice");
    auto finite = [](double v) { return std::isfinite(v); };
    if (!(finite(c->W) && c->W > 0)) return fail(LBM_EINVAL, "W must be > 0");
    if (!finite(c->lambda)) return fail(LBM_EINVAL, "lambda must be finite");
    for (int pi = 0; pi < 2; ++pi)
        for (int a = 0; a < 2; ++a)
            if (!finite(c->c_eq[pi][a])) return fail(LBM_EINVAL, "c_eq must be finite");
    // every BGK rate 1 / (D / c_s^2 + 1/2) must lie in (0, 2): D > 0
    if (!(c->M_phi > 0)) return fail(LBM_EUNSTABLE, "M_phi must be > 0 (rate outside (0, 2))");
    for (int pi = 0; pi < 2; ++pi)
        if (!(c->M_A[pi] > 0) || !(c->M_B[pi] > 0))
            return fail(LBM_EUNSTABLE, "species mobilities must be > 0 (rate outside (0, 2))");
    if (flow) {
        if (!(c->rho0 > 0)) return fail(LBM_EINVAL, "rho0 must be > 0");
        for (int pi = 0; pi < 2; ++pi)
            if (!(c->nu[pi] > 0)) return fail(LBM_EUNSTABLE, "viscosities must be > 0 (rate outside (0, 2))");
        for (double v : {c->drho, c->g[0], c->g[1], c->g[2], c->sigma})
            if (!finite(v)) return fail(LBM_EINVAL, "flow parameters must be finite");
    }
    if (c->ncomp != 0 && c->ncomp != 2 && c->ncomp != 3)
        return fail(LBM_EUNSUPPORTED, "ncomp must be 0 or 2 (the ternary fluid) or 3 (a third composition)");
    const int nc = c->ncomp == 3 ? 3 : 2;
    if (nc == 3) {
        for (int pi = 0; pi < 2; ++pi) {
            if (!finite(c->c_eq_C[pi])) return fail(LBM_EINVAL, "c_eq_C must be finite");
            if (!(c->M_C[pi] > 0)) return fail(LBM_EUNSTABLE, "M_C must be > 0 (rate outside (0, 2))");
        }
        if (c->store_shift_C < -30 || c->store_shift_C > 30)
            return fail(LBM_EINVAL, "store_shift_C out of [-30, 30]");
        if (trt || mrt || vd || gk)
            return fail(LBM_EUNSUPPORTED, "a third composition runs with the BGK Boussinesq step");
        if (paper_scalar)
            return fail(LBM_EUNSUPPORTED, "a third composition runs on the D2Q5 / D3Q7 scalar lattices");
    }
    if (c->precision >= LBM_FP32_FP16STORE)
        for (int i = 0; i < 4; ++i) {
            if (!finite(c->store_ref[i])) return fail(LBM_EINVAL, "store_ref must be finite");
            if (i >= 2 && c->store_ref[i] != 0.0)
                return fail(LBM_EINVAL, "store_ref of h^A, h^B must be 0 (their moving populations have no reference)");
            if (i == 0 && c->precision == LBM_FP32_BF16STORE && c->store_ref[0] != 0.0)
                return fail(LBM_EINVAL, "BF16 storage takes store_ref of f = 0 (f is stored as it is)");
            if (c->store_shift[i] < -30 || c->store_shift[i] > 30)
                return fail(LBM_EINVAL, "store_shift out of [-30, 30]");
        }

    L->prec = c->precision;
    L->qf = c->fluid;
    L->qs = c->scalar;
    L->nc = nc;
    L->nslots = L->qf + (1 + nc) * L->qs;
    L->nodes = nodes;
    if (L->dim == 2) {  // user (x, y) -> kernel (x, z)
        L->NX = c->nx; L->NY = 1; L->NZ = c->ny;
    } else {
        L->NX = c->nx; L->NY = c->ny; L->NZ = c->nz;
    }
    // slots in canonical order; every moving slot takes stride_m bytes, every rest
    // slot stride_r bytes (the kernels rely on this)
    L->stride_m = round_up((size_t)nodes * slot_bytes(L->prec, 1));
    L->stride_r = round_up((size_t)nodes * slot_bytes(L->prec, 0));
    size_t off = 0;
    for (int s = 0; s < L->nslots; ++s) {
        const int k = s < L->qf ? s : (s - L->qf) % L->qs;
        L->slot_off[s] = off;
        off += k == 0 ? L->stride_r : L->stride_m;
    }
    L->copy_bytes = off;

    // kernels and launch geometry: TX x TY node columns marching along z in chunks
    // of zc planes (see below).  Tuning only: the environment variables LBM_TILE
    // ("TXxTY", 2D: "TXx1") and LBM_ZC override the tile and the chunk length.
    int want_tx = 0, want_ty = 0;
    if (const char* e = std::getenv("LBM_TILE")) std::sscanf(e, "%dx%d", &want_tx, &want_ty);
    if (mrt && vd) return fail(LBM_EUNSUPPORTED, "the variable-density model runs with BGK or TRT");
    if (mrt) {
        L->ks = L->dim == 2 ? kernels_mrt_2d(L->qs, L->qf, L->prec) : kernels_mrt_3d(L->qs, L->qf, L->prec);
        if (!L->ks) return fail(LBM_EUNSUPPORTED, "no MRT kernel for this lattice / precision");
    } else if (nc == 3) {
        L->ks = L->dim == 2 ? kernels_nc3_2d(L->qf, L->prec) : kernels_nc3_3d(L->qf, L->prec);
        if (!L->ks) return fail(LBM_EUNSUPPORTED, "no kernel with a third composition for this lattice / precision");
    } else if (gk) {
        L->ks = L->dim == 2 ? kernels_gk_2d(L->qs, L->qf, L->prec) : kernels_gk_3d(L->qs, L->qf, L->prec);
        if (!L->ks) return fail(LBM_EUNSUPPORTED, "no general_kappa kernel for this lattice / precision");
    } else if (vd) {
        L->ks = L->dim == 2 ? kernels_vd_2d(L->qs, trt, L->prec) : kernels_vd_3d(L->qs, trt, L->prec);
        if (!L->ks) return fail(LBM_EUNSUPPORTED, "no variable-density kernel for this lattice / precision");
    } else if (trt) {
        L->ks = L->dim == 2 ? kernels_trt_2d(L->qs, L->qf, L->prec) : kernels_trt_3d(L->qs, L->qf, L->prec);
        if (!L->ks) return fail(LBM_EUNSUPPORTED, "no TRT kernel for this lattice / precision");
    } else if (paper_scalar) {
        L->ks = L->dim == 2 ? kernels_paper_2d(L->qf, L->prec) : kernels_paper_3d(L->qf, L->prec);
        if (!L->ks) return fail(LBM_EUNSUPPORTED, "no kernel for the D2Q9 / D3Q19 scalar lattices at this precision");
    } else {
        L->ks = L->dim == 2 ? kernels_2d(L->qf, L->prec, want_tx) : kernels_3d(L->qf, L->prec, want_tx, want_ty);
    }
    if (!L->ks) return fail(LBM_EUNSUPPORTED, "no kernel for this lattice / precision");
    L->tx = L->ks->tx;
    L->ty = L->ks->ty;
    const long long gx = (L->NX + L->tx - 1) / L->tx, gy = (L->NY + L->ty - 1) / L->ty;
    const long long cols = std::max(1LL, gx * gy);
    long long nchunks;
    if (L->dim == 2) {
        // rows of TX nodes: about 2048 work-groups (8 per compute unit); a 512^2 box then
        // takes one or two rows per group, the fastest on one MI355X (measured)
        nchunks = 2048 / cols;
    } else {
        // 3D columns: measured on one MI355X (256 compute units), the step is fastest when
        // all of its work-groups are resident at once, with two per compute unit for
        // FP32 / FP64 storage (HBM-bound: 15.2 GLUPS at 256^3 against 14.5 with 2048
        // groups) and three for 16-bit storage (instruction-bound: 21.4 against 20.5);
        // when the columns alone exceed that, with 64-plane chunks (512^3 BF16: 20.9
        // GLUPS against 20.0 with 256-plane chunks).  Equal chunks: zc divides nz evenly
        // when it can.  The layout depends only on the configuration, never on the device.
        constexpr long long kCUs = 256;
        const long long per_cu = (L->prec == LBM_FP32 || L->prec == LBM_FP64) ? 2 : 3;
        nchunks = cols <= per_cu * kCUs ? (per_cu * kCUs) / cols : (L->NZ + 63) / 64;
    }
    nchunks = std::max(1LL, std::min<long long>(L->NZ, nchunks));
    int zc = int((L->NZ + nchunks - 1) / nchunks);
    if (const char* e = std::getenv("LBM_ZC")) {
        const int v = std::atoi(e);
        if (v > 0) zc = std::min(v, L->NZ);
    }
    L->zc = zc;
    const long long gz = (L->NZ + zc - 1) / zc;
    L->tiles[0] = int(gx); L->tiles[1] = int(gy); L->tiles[2] = int(gz);
    L->grid = dim3(unsigned(gx * gy * gz));
    L->nparts = gx * gy * gz;
    // aux: kAuxHead doubles of scalars, then per-work-group partials (8 per group
    // of the fused kernel, 9 with a third composition; one per group of the Euler
    // characteristic, <= 1024)
    const long long npart_doubles = std::max<long long>((nc == 3 ? 9 : 8) * L->nparts, 1024);
    L->aux_bytes = round_up(sizeof(double) * (kAuxHead + npart_doubles));
    L->mask_off = 2 * L->copy_bytes + L->aux_bytes;
    L->state_bytes = L->mask_off + round_up((size_t)nodes);
    L->adj_stride = round_up((size_t)nodes * 4);
    L->aux_stride_elems = round_up((size_t)nodes * 4) / 4;
    L->adj_parts = (nodes + 255) / 256;
    // adjoint state first (two lambda copies, the c_F rows), then the per-step scratch
    L->adj_state_bytes = 2 * L->nslots * L->adj_stride + kAuxCRows * L->aux_stride_elems * 4;
    L->adj_scratch_bytes = kAuxRows * L->aux_stride_elems * 4 + round_up(sizeof(double) * 6 * L->adj_parts) +
                           round_up((size_t)nodes * sizeof(double));
    L->adj_bytes = L->adj_state_bytes + L->adj_scratch_bytes;
    return LBM_OK;
}

}  // namespace

struct lbm_handle {
    lbm_config cfg;
    Layout L;
    const KernelSet* ks;
    char* copy[2];
    double* aux;
    unsigned char* mask;
    int cur;
    int64_t steps;
    int adj_cur;   // adjoint copy holding the current lambda (in the caller's workspace)
    KParams base;  // every field except src/dst/mout
    // the initial fields given to lbm_init (caller-owned), for lbm_init_adjoint
    const double* phi0;
    const double* muA0;
    const double* muB0;
    bool given_c;  // made by lbm_init_composition
};

namespace {

void set_slots(const lbm_handle* h, KParams& kp, const char* src, char* dst) {
    kp.src_base = src;
    kp.dst_base = dst;
    for (int s = 0; s < kMaxSlots; ++s) {
        const bool used = s < h->L.nslots;
        kp.src_slot[s] = (src && used) ? src + h->L.slot_off[s] : nullptr;
        kp.dst_slot[s] = (dst && used) ? dst + h->L.slot_off[s] : nullptr;
    }
}

void fill_params(lbm_handle* h) {
    const lbm_config& c = h->cfg;
    const Layout& L = h->L;
    KParams& kp = h->base;
    std::memset(&kp, 0, sizeof(kp));
    kp.nx = L.NX; kp.ny = L.NY; kp.nz = L.NZ;
    if (L.dim == 2) {
        kp.wall_x = c.bc[0] == LBM_WALLS; kp.wall_y = 0; kp.wall_z = c.bc[1] == LBM_WALLS;
        kp.gx = c.g[0]; kp.gy = 0.0; kp.gz = c.g[1];
    } else {
        kp.wall_x = c.bc[0] == LBM_WALLS; kp.wall_y = c.bc[1] == LBM_WALLS; kp.wall_z = c.bc[2] == LBM_WALLS;
        kp.gx = c.g[0]; kp.gy = c.g[1]; kp.gz = c.g[2];
    }
    kp.zc = L.zc;
    kp.tiles_x = L.tiles[0]; kp.tiles_y = L.tiles[1]; kp.tiles_z = L.tiles[2];
    kp.mean_subtract = c.gravity_mean_subtract ? 1 : 0;
    kp.W = c.W;
    kp.lam = c.lambda;
    kp.mphi_w2 = c.M_phi / (c.W * c.W);
    kp.c0A = c.c_eq[0][0]; kp.c0B = c.c_eq[0][1];
    kp.c1A = c.c_eq[1][0]; kp.c1B = c.c_eq[1][1];
    // c_s^2 of the scalar lattice
    const double cs2s = L.qs == 5 ? D2Q5K::cs2 : L.qs == 7 ? D3Q7K::cs2 : L.qs == 9 ? D2Q9K::cs2 : D3Q19K::cs2;
    kp.omega_g = 1.0 / (c.M_phi / cs2s + 0.5);
    // TRT: the symmetric rate of g from Lambda_s = (1/w+ - 1/2)(1/w- - 1/2), w- = omega_g
    kp.trt_lf = c.trt_magic[0];
    kp.trt_ls = c.trt_magic[1];
    kp.omega_gp = c.collision == LBM_TRT ? 1.0 / (0.5 + c.trt_magic[1] / (c.M_phi / cs2s)) : kp.omega_g;
    kp.f32.trt_lf = float(kp.trt_lf);
    kp.f32.trt_ls = float(kp.trt_ls);
    kp.f32.omega_gp = float(kp.omega_gp);
    kp.variable_density = c.variable_density;
    kp.general_k = c.general_kappa;
    for (int i = 0; i < 3; ++i) {
        kp.mrt_f[i] = c.mrt_rates[0][i];
        kp.mrt_s[i] = c.mrt_rates[1][i];
        kp.f32.mrt_f[i] = float(kp.mrt_f[i]);
        kp.f32.mrt_s[i] = float(kp.mrt_s[i]);
    }
    for (int i = 0; i < 3; ++i) {
        kp.kap0[i] = c.general_kappa ? c.kappa[0][i] : (i == 1 ? 0.0 : 1.0);
        kp.kap1[i] = c.general_kappa ? c.kappa[1][i] : (i == 1 ? 0.0 : 1.0);
    }
    kp.MA0 = c.M_A[0]; kp.MA1 = c.M_A[1]; kp.MB0 = c.M_B[0]; kp.MB1 = c.M_B[1];
    if (L.nc == 3) {
        kp.c0C = c.c_eq_C[0]; kp.c1C = c.c_eq_C[1];
        kp.MC0 = c.M_C[0]; kp.MC1 = c.M_C[1];
    }
    kp.f32.MC0 = float(kp.MC0);
    kp.f32.MC1 = float(kp.MC1);
    kp.nu0 = c.nu[0]; kp.nu1 = c.nu[1];
    kp.rho0 = L.qf ? c.rho0 : 1.0;
    kp.drho = c.drho;
    kp.cap = 1.5 * c.sigma * c.W;
    kp.inv_W2 = 1.0 / (c.W * c.W);
    kp.dK_dW = -2.0 * c.M_phi / (c.W * c.W * c.W);
    kp.dcap_dW = 1.5 * c.sigma;
    kp.f32.cap = float(kp.cap);
    kp.f32.inv_W2 = float(kp.inv_W2);
    kp.f32.drho = float(kp.drho);
    kp.f32.gx = float(kp.gx);
    kp.f32.gy = float(kp.gy);
    kp.f32.gz = float(kp.gz);
    kp.f32.inv_rho0 = float(1.0 / kp.rho0);
    kp.f32.rho0 = float(kp.rho0);
    kp.f32.nu0 = float(kp.nu0);
    kp.f32.nu1 = float(kp.nu1);
    kp.f32.omega_g = float(kp.omega_g);
    kp.f32.MA0 = float(kp.MA0);
    kp.f32.MA1 = float(kp.MA1);
    kp.f32.MB0 = float(kp.MB0);
    kp.f32.MB1 = float(kp.MB1);
    const bool sixteen = L.prec == LBM_FP32_FP16STORE || L.prec == LBM_FP32_BF16STORE;
    for (int f = 0; f < 5; ++f) {
        // BF16 has the exponent range of FP32: its deviations are stored unscaled.
        // Field 4 (h^C) takes reference 0, as h^A and h^B
        const int shf = f < 4 ? c.store_shift[f] : (L.nc == 3 ? c.store_shift_C : 0);
        const int sh = L.prec == LBM_FP32_FP16STORE ? shf : 0;
        kp.fref[f] = (sixteen && f < 4) ? float(c.store_ref[f]) : 0.0f;
        kp.fscale[f] = std::ldexp(1.0f, sh);
        kp.finv[f] = std::ldexp(1.0f, -sh);
    }
    kp.stride_m = L.stride_m;
    kp.stride_r = L.stride_r;
    kp.phi_ref = h->aux;
    kp.partials = h->aux + kAuxHead;
}

int check_handle(const lbm_handle* h) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    return LBM_OK;
}

int launched(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LBM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

int lbm_state_bytes(const lbm_config* cfg, size_t* bytes) {
    Layout L;
    if (int r = check_config(cfg, &L)) return r;
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    *bytes = L.state_bytes;
    return LBM_OK;
}

int lbm_checkpoint_bytes(const lbm_config* cfg, size_t* bytes) {
    Layout L;
    if (int r = check_config(cfg, &L)) return r;
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    *bytes = L.copy_bytes + kAlign;
    return LBM_OK;
}

namespace {

int scratch_for_current_device(void** out);  // the scratch of lbm_adjoint_step_noalloc

// mu[a], c[a]: potential and (optional) composition of composition a (A, B, C)
int init_impl(const lbm_config* cfg, void* state, size_t state_bytes, const double* phi0, const double* const* c,
              const double* const* mu, int nc_given, void* stream, lbm_handle** out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    if (int r = check_config(cfg, &L)) return r;
    if (nc_given != L.nc)
        return fail(LBM_EINVAL, L.nc == 3 ? "a configuration with ncomp = 3 is initialised with lbm_init_multi"
                                          : "lbm_init_multi got a different number of compositions");
    if (!state || !phi0) return fail(LBM_EINVAL, "NULL device pointer");
    for (int a = 0; a < L.nc; ++a)
        if (!mu[a]) return fail(LBM_EINVAL, "NULL device pointer");
    for (int a = 1; a < L.nc; ++a)
        if ((c[a] == nullptr) != (c[0] == nullptr)) return fail(LBM_EINVAL, "give every composition or none");
    const double* cA0 = c[0];
    const double* muA0 = mu[0];
    const double* muB0 = mu[1];
    if ((reinterpret_cast<uintptr_t>(state) % kAlign) != 0)
        return fail(LBM_EINVAL, "state must be 256-byte aligned");
    if (state_bytes < L.state_bytes)
        return fail(LBM_ESIZE, "state buffer smaller than lbm_state_bytes");
    const KernelSet* ks = L.ks;

    lbm_handle* h = new lbm_handle();
    h->cfg = *cfg;
    h->L = L;
    h->ks = ks;
    h->copy[0] = static_cast<char*>(state);
    h->copy[1] = static_cast<char*>(state) + L.copy_bytes;
    h->aux = reinterpret_cast<double*>(static_cast<char*>(state) + 2 * L.copy_bytes);
    h->mask = reinterpret_cast<unsigned char*>(static_cast<char*>(state) + L.mask_off);
    h->cur = 0;
    h->steps = 0;
    h->adj_cur = 0;
    h->phi0 = phi0;
    h->muA0 = muA0;
    h->muB0 = muB0;
    h->given_c = cA0 != nullptr;
    fill_params(h);
    hipStream_t s = static_cast<hipStream_t>(stream);

    auto bail = [&](int r) { delete h; return r; };
    {
        // set-up of the no-alloc adjoint step's scratch on this device (once per device)
        void* t = nullptr;
        if (int r = scratch_for_current_device(&t)) return bail(r);
    }
    if (hipMemsetAsync(h->aux, 0, kAuxHead * sizeof(double), s) != hipSuccess)
        return bail(fail(LBM_EHIP, "hipMemsetAsync of the aux area failed"));
    // both population copies start zeroed: the padding after each slot is then zero for
    // good (no kernel writes it), and so are the padding bytes of every checkpoint
    launch_zero(reinterpret_cast<double*>(h->copy[0]), (long long)(2 * L.copy_bytes / sizeof(double)), s);
    if (cfg->gravity_mean_subtract) {
        // <phi_0> for the buoyancy reference of the first step
        const int nb = int(std::min<long long>(1024, (L.nodes + 255) / 256));
        launch_sum_partials(phi0, L.nodes, h->aux + kAuxHead, nb, s);
        launch_finalize(h->aux + kAuxHead, nb, 1, -1, 1.0 / double(L.nodes), h->aux, s);
        if (int r = launched("phi_0 mean")) return bail(r);
    }
    KParams kp = h->base;
    set_slots(h, kp, nullptr, h->copy[0]);
    for (int a = 0; a < L.nc; ++a) kp.init_c[a] = c[a];
    ks->init(kp, phi0, muA0, muB0, L.nc == 3 ? mu[2] : nullptr, s);
    if (int r = launched("init kernel")) return bail(r);
    *out = h;
    return LBM_OK;
}

}  // namespace

int lbm_init(const lbm_config* cfg, void* state, size_t state_bytes, const double* phi0,
             const double* muA0, const double* muB0, void* stream, lbm_handle** out) {
    const double* c[3] = {nullptr, nullptr, nullptr};
    const double* mu[3] = {muA0, muB0, nullptr};
    return init_impl(cfg, state, state_bytes, phi0, c, mu, 2, stream, out);
}

int lbm_init_multi(const lbm_config* cfg, void* state, size_t state_bytes, const double* phi0,
                   const double* const* mu0, const double* const* c0, void* stream, lbm_handle** out) {
    if (out) *out = nullptr;
    if (!cfg) return fail(LBM_EINVAL, "config is NULL");
    if (!mu0) return fail(LBM_EINVAL, "mu0 is NULL");
    const int nc = cfg->ncomp == 3 ? 3 : 2;
    const double* c[3] = {nullptr, nullptr, nullptr};
    const double* mu[3] = {nullptr, nullptr, nullptr};
    for (int a = 0; a < nc; ++a) {
        mu[a] = mu0[a];
        c[a] = c0 ? c0[a] : nullptr;
        if (c0 && !c0[a]) return fail(LBM_EINVAL, "NULL device pointer");
    }
    return init_impl(cfg, state, state_bytes, phi0, c, mu, nc, stream, out);
}

int lbm_init_composition(const lbm_config* cfg, void* state, size_t state_bytes, const double* phi0,
                         const double* cA0, const double* cB0, const double* muA0, const double* muB0,
                         void* stream, lbm_handle** out) {
    if (!cA0 || !cB0) {
        if (out) *out = nullptr;
        return fail(LBM_EINVAL, "NULL device pointer");
    }
    const double* c[3] = {cA0, cB0, nullptr};
    const double* mu[3] = {muA0, muB0, nullptr};
    return init_impl(cfg, state, state_bytes, phi0, c, mu, 2, stream, out);
}

int lbm_step(lbm_handle* h, int64_t nsteps, void* stream) {
    if (int r = check_handle(h)) return r;
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    KParams kp[2] = {h->base, h->base};
    set_slots(h, kp[0], h->copy[0], h->copy[1]);
    set_slots(h, kp[1], h->copy[1], h->copy[0]);
    // walls on x and y: the fix-up kernel; z walls bounce back when the next step pulls
    const int walls[2] = {h->base.wall_x, h->base.wall_y};
    for (int64_t i = 0; i < nsteps; ++i) {
        h->ks->fused(MODE_STEP, h->L.grid, kp[h->cur], s);
        for (int a = 0; a < 2; ++a)
            if (walls[a]) h->ks->walls(kp[h->cur], a, s);
        if (h->cfg.gravity_mean_subtract)
            launch_finalize(h->aux + kAuxHead, int(h->L.nparts), 1, -1, 1.0 / double(h->L.nodes), h->aux, s);
        if (int r = launched("step kernel")) return r;
        h->cur ^= 1;
        h->steps += 1;
    }
    return LBM_OK;
}

int lbm_moments(lbm_handle* h, uint32_t mask, void* const* out, int32_t out_dtype, void* stream) {
    if (int r = check_handle(h)) return r;
    if (out_dtype != LBM_OUT_F64 && out_dtype != LBM_OUT_F32) return fail(LBM_EINVAL, "bad out_dtype");
    if (mask >> LBM_NMOM) return fail(LBM_EINVAL, "unknown bits in mask");
    if (mask && !out) return fail(LBM_EINVAL, "out is NULL");
    for (int i = 0; i < LBM_NMOM; ++i)
        if ((mask >> i & 1u) && !out[i]) return fail(LBM_EINVAL, "NULL output for a requested moment");
    hipStream_t s = static_cast<hipStream_t>(stream);
    KParams kp = h->base;
    set_slots(h, kp, h->copy[h->cur], nullptr);
    for (int i = 0; i < kNumMom; ++i) kp.mout[i] = nullptr;
    if ((mask & (LBM_M_CC | LBM_M_MUC)) && h->L.nc != 3)
        return fail(LBM_EINVAL, "LBM_M_CC / LBM_M_MUC need a third composition (ncomp = 3)");
    for (int i = 0; i < 6; ++i)
        if (mask >> i & 1u) kp.mout[i] = out[i];
    for (int i = 9; i < 11; ++i)
        if (mask >> i & 1u) kp.mout[i] = out[i];
    const size_t esize = out_dtype == LBM_OUT_F32 ? 4 : 8;
    if (h->L.dim == 3) {
        for (int i = 6; i < 9; ++i)
            if (mask >> i & 1u) kp.mout[i] = out[i];
    } else {
        if (mask & LBM_M_UX) kp.mout[6] = out[6];
        if (mask & LBM_M_UY) kp.mout[8] = out[7];  // user y is the kernel z axis
        if (mask & LBM_M_UZ) LBM_HIP(hipMemsetAsync(out[8], 0, esize * h->L.nodes, s));
    }
    kp.mout_f32 = out_dtype == LBM_OUT_F32;
    if (mask) {
        h->ks->fused(MODE_MOMENTS, h->L.grid, kp, s);
        if (int r = launched("moments kernel")) return r;
    }
    return LBM_OK;
}

namespace {

EulerGeom euler_geometry(const lbm_handle* h) {
    const Layout& L = h->L;
    const KParams& b = h->base;
    EulerGeom g{};
    const long long sx = 1, sy = L.NX, sz = (long long)L.NX * L.NY;
    auto add = [&](int n, int wall, long long stride) {
        g.n[g.d] = n; g.wall[g.d] = wall; g.stride[g.d] = stride; ++g.d;
    };
    add(L.NX, b.wall_x, sx);
    if (L.dim == 2) {
        add(L.NZ, b.wall_z, sz);  // user y
    } else {
        add(L.NY, b.wall_y, sy);
        if (L.NZ > 1) add(L.NZ, b.wall_z, sz);
    }
    g.nanchors = 1;
    for (int a = 0; a < g.d; ++a) g.nanchors *= g.n[a] + g.wall[a];
    return g;
}

}  // namespace

int lbm_diagnostics(lbm_handle* h, double* host_out, void* stream) {
    if (int r = check_handle(h)) return r;
    if (!host_out) return fail(LBM_EINVAL, "host_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    KParams kp = h->base;
    set_slots(h, kp, h->copy[h->cur], nullptr);
    kp.mask_out = h->mask;
    h->ks->fused(MODE_DIAG, h->L.grid, kp, s);
    // 8 reductions (9 with a third composition: sum c^C goes to LBM_D_SUM_CC)
    launch_finalize(h->aux + kAuxHead, int(h->L.nparts), h->L.nc == 3 ? 9 : 8, 4, 1.0, h->aux + 8, s);
    // droplet count: Euler characteristic of the cells with phi >= 1/2, over the
    // axes of the run (2D runs: user x and y; 3D runs with nz = 1 count as 2D)
    const EulerGeom g = euler_geometry(h);
    const int nb = int(std::min<long long>(1024, (g.nanchors + 255) / 256));
    launch_euler(h->mask, g, h->aux + kAuxHead, nb, s);
    launch_finalize(h->aux + kAuxHead, nb, 1, -1, 1.0, h->aux + 8 + LBM_D_DROPLETS, s);
    if (int r = launched("diagnostics kernels")) return r;
    // entries 0 .. LBM_NDIAG - 1 (the mean radius is set below; sum c^C stays 0 without
    // a third composition: the aux head is zeroed at initialisation)
    LBM_HIP(hipMemcpyAsync(host_out, h->aux + 8, LBM_NDIAG * sizeof(double), hipMemcpyDeviceToHost, s));
    LBM_HIP(hipStreamSynchronize(s));
    // mean radius from the interface integral I (Eq. Rmoy_2D, I = 2 pi N <R>; in 3D
    // spheres: I = 4 pi N <R>^2)
    const double I = host_out[LBM_D_INTERFACE], N = host_out[LBM_D_DROPLETS];
    const double pi = 3.14159265358979323846;
    host_out[LBM_D_MEAN_RADIUS] = N <= 0 ? 0.0 : (g.d == 2 ? I / (2 * pi * N) : std::sqrt(I / (4 * pi * N)));
    return LBM_OK;
}

int lbm_run_series(lbm_handle* h, int64_t nsteps, int64_t every, double* host_out, void* stream) {
    if (int r = check_handle(h)) return r;
    if (!host_out) return fail(LBM_EINVAL, "host_out is NULL");
    if (every < 1 || nsteps < 0 || nsteps % every != 0)
        return fail(LBM_EINVAL, "nsteps must be a non-negative multiple of every >= 1");
    const int64_t rows = nsteps / every + 1;
    for (int64_t i = 0; i < rows; ++i) {
        if (i > 0)
            if (int r = lbm_step(h, every, stream)) return r;
        if (int r = lbm_diagnostics(h, host_out + i * LBM_NDIAG, stream)) return r;
    }
    return LBM_OK;
}

int lbm_get_populations(lbm_handle* h, double* dst, void* stream) {
    if (int r = check_handle(h)) return r;
    if (!dst) return fail(LBM_EINVAL, "dst is NULL");
    KParams kp = h->base;
    set_slots(h, kp, h->copy[h->cur], nullptr);
    h->ks->get_pops(kp, h->L.nslots, h->L.nodes, dst, static_cast<hipStream_t>(stream));
    return launched("get_populations kernel");
}

int lbm_set_populations(lbm_handle* h, const double* src, void* stream) {
    if (int r = check_handle(h)) return r;
    if (!src) return fail(LBM_EINVAL, "src is NULL");
    KParams kp = h->base;
    set_slots(h, kp, nullptr, h->copy[h->cur]);
    h->ks->set_pops(kp, h->L.nslots, h->L.nodes, src, static_cast<hipStream_t>(stream));
    return launched("set_populations kernel");
}

namespace {

// the bytes of a checkpoint after the buffered <phi>: zero, so that a checkpoint is a
// function of the state alone (a fill kernel, not a memset: callers may capture it)
int zero_tail(const lbm_handle* h, void* ckpt, hipStream_t s) {
    char* tail = static_cast<char*>(ckpt) + h->L.copy_bytes + sizeof(double);
    constexpr long long n = (kAlign - sizeof(double)) / sizeof(double);
    if (reinterpret_cast<uintptr_t>(tail) % alignof(double) == 0) {
        launch_zero(reinterpret_cast<double*>(tail), n, s);
        return launched("checkpoint tail");
    }
    LBM_HIP(hipMemsetAsync(tail, 0, kAlign - sizeof(double), s));
    return LBM_OK;
}

}  // namespace

int lbm_save(lbm_handle* h, void* dst, void* stream) {
    if (int r = check_handle(h)) return r;
    if (!dst) return fail(LBM_EINVAL, "dst is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    LBM_HIP(hipMemcpyAsync(dst, h->copy[h->cur], h->L.copy_bytes, hipMemcpyDeviceToDevice, s));
    LBM_HIP(hipMemcpyAsync(static_cast<char*>(dst) + h->L.copy_bytes, h->aux, sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    return zero_tail(h, dst, s);
}

int lbm_restore(lbm_handle* h, const void* src, void* stream) {
    if (int r = check_handle(h)) return r;
    if (!src) return fail(LBM_EINVAL, "src is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    LBM_HIP(hipMemcpyAsync(h->copy[h->cur], src, h->L.copy_bytes, hipMemcpyDeviceToDevice, s));
    LBM_HIP(hipMemcpyAsync(h->aux, static_cast<const char*>(src) + h->L.copy_bytes, sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    return LBM_OK;
}

int lbm_set_state(lbm_handle* h, const void* src, void* stream) { return lbm_restore(h, src, stream); }

int lbm_adjoint_bytes(const lbm_config* cfg, size_t* bytes) {
    Layout L;
    if (int r = check_config(cfg, &L)) return r;
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    *bytes = L.adj_bytes;
    return LBM_OK;
}

int lbm_step_external(lbm_handle* h, const void* src, void* dst, void* phi_src, void* stream) {
    if (int r = check_handle(h)) return r;
    if (!src || !dst || src == dst) return fail(LBM_EINVAL, "src and dst must be distinct checkpoint buffers");
    hipStream_t s = static_cast<hipStream_t>(stream);
    KParams kp = h->base;
    set_slots(h, kp, static_cast<const char*>(src), static_cast<char*>(dst));
    kp.phi_out = phi_src;
    const double* ref_in = reinterpret_cast<const double*>(static_cast<const char*>(src) + h->L.copy_bytes);
    double* ref_out = reinterpret_cast<double*>(static_cast<char*>(dst) + h->L.copy_bytes);
    kp.phi_ref = ref_in;
    // the buffered <phi> is recomputed with the mean subtraction, else carried over
    kp.ref_copy = h->cfg.gravity_mean_subtract ? nullptr : ref_out;
    h->ks->fused(phi_src ? MODE_STEP_PHI : MODE_STEP, h->L.grid, kp, s);
    const int walls[2] = {h->base.wall_x, h->base.wall_y};
    for (int a = 0; a < 2; ++a)
        if (walls[a]) h->ks->walls(kp, a, s);
    if (h->cfg.gravity_mean_subtract)
        launch_finalize(h->aux + kAuxHead, int(h->L.nparts), 1, -1, 1.0 / double(h->L.nodes), ref_out, s);
    return launched("step_external kernels");
}

int lbm_phase_field(lbm_handle* h, const void* state, void* phi, void* stream) {
    if (int r = check_handle(h)) return r;
    if (!state || !phi) return fail(LBM_EINVAL, "NULL pointer");
    KParams kp = h->base;
    set_slots(h, kp, static_cast<const char*>(state), nullptr);
    kp.phi_ref = reinterpret_cast<const double*>(static_cast<const char*>(state) + h->L.copy_bytes);
    for (int i = 0; i < kNumMom; ++i) kp.mout[i] = nullptr;
    kp.mout[0] = phi;
    kp.mout_f32 = h->L.prec == LBM_FP64 ? 0 : 1;
    h->ks->fused(MODE_MOMENTS, h->L.grid, kp, static_cast<hipStream_t>(stream));
    return launched("phase-field kernel");
}

namespace {

int adjoint_ready(const lbm_handle* h, const void* work) {
    if (int r = check_handle(h)) return r;
    if (!work) return fail(LBM_EINVAL, "work is NULL");
    if (!h->ks->adj_step)
        return fail(LBM_EUNSUPPORTED, "the adjoint runs on FP32 or FP64 storage with the BGK Boussinesq model");
    if (h->cfg.gravity_mean_subtract)
        return fail(LBM_EUNSUPPORTED, "the adjoint does not support gravity_mean_subtract");
    return LBM_OK;
}

// workspace pieces
struct AdjWork {
    char* lam[2];
    float* auxc;    // c_F rows (adjoint state)
    float* aux;     // per-step scratch rows
    double* part;   // ceil(nodes / 256) x 6, indexed by work-group of the node kernels
    long long nparts;
    void* phi;      // phi of a state ([node], the compute type)
};

// the pieces of an adjoint state buffer `state` and a scratch area `scratch` (which
// directly follows the state in an lbm_adjoint_bytes workspace)
AdjWork adjoint_parts(const lbm_handle* h, void* state, void* scratch) {
    char* w = static_cast<char*>(state);
    const size_t copy = h->L.nslots * h->L.adj_stride, row = h->L.aux_stride_elems * 4;
    AdjWork a;
    a.lam[0] = w;
    a.lam[1] = w + copy;
    a.auxc = reinterpret_cast<float*>(w + 2 * copy);
    char* t = static_cast<char*>(scratch);
    a.aux = reinterpret_cast<float*>(t);
    a.part = reinterpret_cast<double*>(t + kAuxRows * row);
    a.nparts = h->L.adj_parts;
    a.phi = t + kAuxRows * row + round_up(sizeof(double) * 6 * a.nparts);
    return a;
}

AdjWork adjoint_work(const lbm_handle* h, void* work) {
    return adjoint_parts(h, work, static_cast<char*>(work) + h->L.adj_state_bytes);
}

// adjoint fields of a KParams: lambda copy `in` -> `out`
void adjoint_params(const lbm_handle* h, KParams& kp, const AdjWork& a, int in, int out) {
    kp.adj_in = in >= 0 ? a.lam[in] : nullptr;
    kp.adj_out = out >= 0 ? a.lam[out] : nullptr;
    kp.adj_stride = h->L.adj_stride;
    kp.aux = a.aux;
    kp.auxc = a.auxc;
    kp.aux_stride = h->L.aux_stride_elems;
    kp.partials = a.part;
}

void zero_partials(const AdjWork& a, hipStream_t s) { launch_zero(a.part, 6 * a.nparts, s); }

}  // namespace

int lbm_adjoint_seed(lbm_handle* h, const void* state, const double* dL_dphi, void* work, void* stream) {
    if (int r = adjoint_ready(h, work)) return r;
    if (!state || !dL_dphi) return fail(LBM_EINVAL, "NULL pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const AdjWork a = adjoint_work(h, work);
    zero_partials(a, s);
    KParams kp = h->base;
    set_slots(h, kp, static_cast<const char*>(state), nullptr);
    adjoint_params(h, kp, a, -1, 0);
    h->ks->adj_seed(kp, h->L.nodes, dL_dphi, s);
    h->adj_cur = 0;
    return launched("adjoint seed kernels");
}

namespace {

// node and gather kernels of one adjoint step on the pieces `a`, phi of the state given
int adjoint_step_parts(lbm_handle* h, const void* state, const void* phi, const AdjWork& a, hipStream_t s) {
    KParams kp = h->base;
    set_slots(h, kp, static_cast<const char*>(state), nullptr);
    kp.phi_ref = reinterpret_cast<const double*>(static_cast<const char*>(state) + h->L.copy_bytes);
    adjoint_params(h, kp, a, h->adj_cur, 1 - h->adj_cur);
    h->ks->adj_step(kp, h->L.nodes, phi, s);
    h->ks->adj_gather(kp, h->L.nodes, 0, nullptr, s);
    h->adj_cur = 1 - h->adj_cur;
    return launched("adjoint step kernels");
}

}  // namespace

int lbm_adjoint_step_phi(lbm_handle* h, const void* state, const void* phi, void* work, void* stream) {
    if (int r = adjoint_ready(h, work)) return r;
    if (!state || !phi) return fail(LBM_EINVAL, "NULL pointer");
    return adjoint_step_parts(h, state, phi, adjoint_work(h, work), static_cast<hipStream_t>(stream));
}

int lbm_adjoint_step(lbm_handle* h, const void* state_n, void* adj_inout, double* grad_params, void* stream) {
    if (int r = adjoint_ready(h, adj_inout)) return r;
    if (!state_n || !grad_params) return fail(LBM_EINVAL, "NULL pointer");
    const AdjWork a = adjoint_work(h, adj_inout);
    // phi of state n, the field the step's stencil used (Eq. Moment0_Phi)
    if (int r = lbm_phase_field(h, state_n, a.phi, stream)) return r;
    if (int r = lbm_adjoint_step_phi(h, state_n, a.phi, adj_inout, stream)) return r;
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_sum6(a.part, int(a.nparts), grad_params, true, s);
    zero_partials(a, s);
    return launched("adjoint parameter reduction");
}

// ---- the adjoint step for callers that cannot allocate ----------------------------
// Its per-step scratch (kAuxRows rows, theta partials, phi of the state) lives in a
// file-scope device array of kNoallocScratch bytes, one per GPU, kept until the
// process ends.  Host code takes the array's device address per device with
// hipGetSymbolAddress (the array's name is a host-side stand-in, not that address).

namespace {

constexpr size_t kNoallocScratch = size_t(32) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoallocScratch];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// the scratch array's address on the current device (looked up once per device)
int scratch_for_current_device(void** out) {
    int dev = -1;
    LBM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EHIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        LBM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

}  // namespace

int lbm_adjoint_step_noalloc(lbm_handle* h, const void* state_n, void* adj_state, double* grad_params,
                             void* stream) {
    if (int r = adjoint_ready(h, adj_state)) return r;
    if (!state_n || !grad_params) return fail(LBM_EINVAL, "NULL pointer");
    if (h->L.adj_scratch_bytes > kNoallocScratch)
        return fail(LBM_ESIZE, "grid too large for the 32 MiB scratch of lbm_adjoint_step_noalloc "
                               "(about 36 bytes per node)");
    void* t = nullptr;
    if (int r = scratch_for_current_device(&t)) return r;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const AdjWork a = adjoint_parts(h, adj_state, t);
    // the scratch keeps the previous call's contents: clear it (a kernel, no memset)
    launch_zero(reinterpret_cast<double*>(t), (long long)(h->L.adj_scratch_bytes / sizeof(double)), s);
    if (int r = lbm_phase_field(h, state_n, a.phi, stream)) return r;
    if (int r = adjoint_step_parts(h, state_n, a.phi, a, s)) return r;
    launch_sum6(a.part, int(a.nparts), grad_params, true, s);
    return launched("adjoint parameter reduction");
}

int lbm_adjoint_init(lbm_handle* h, const double* phi0, const double* muA0, const double* muB0, void* work,
                     double* grad_phi0, void* stream) {
    if (int r = adjoint_ready(h, work)) return r;
    if (!phi0 || !muA0 || !muB0 || !grad_phi0) return fail(LBM_EINVAL, "NULL pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const AdjWork a = adjoint_work(h, work);
    KParams kp = h->base;
    adjoint_params(h, kp, a, h->adj_cur, -1);
    h->ks->adj_init_local(kp, h->L.nodes, phi0, muA0, muB0, s);
    h->ks->adj_gather(kp, h->L.nodes, 1, grad_phi0, s);
    return launched("adjoint init kernels");
}

int lbm_init_adjoint(lbm_handle* h, const void* adj_state0, double* grad_phi0, double* grad_params, void* stream) {
    if (int r = adjoint_ready(h, adj_state0)) return r;
    if (!grad_phi0 || !grad_params) return fail(LBM_EINVAL, "NULL pointer");
    if (h->given_c)
        return fail(LBM_EUNSUPPORTED, "the adjoint of the initialisation needs the closure's compositions (lbm_init)");
    void* work = const_cast<void*>(adj_state0);
    if (int r = lbm_adjoint_init(h, h->phi0, h->muA0, h->muB0, work, grad_phi0, stream)) return r;
    const AdjWork a = adjoint_work(h, work);
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_sum6(a.part, int(a.nparts), grad_params, true, s);
    zero_partials(a, s);
    return launched("adjoint parameter reduction");
}

int lbm_adjoint_theta(lbm_handle* h, void* work, double* grad_theta, void* stream) {
    if (int r = adjoint_ready(h, work)) return r;
    if (!grad_theta) return fail(LBM_EINVAL, "grad_theta is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const AdjWork a = adjoint_work(h, work);
    launch_sum6(a.part, int(a.nparts), grad_theta, false, s);
    return launched("adjoint parameter reduction");
}

int lbm_adjoint_get(lbm_handle* h, void* work, double* dst, void* stream) {
    if (int r = adjoint_ready(h, work)) return r;
    if (!dst) return fail(LBM_EINVAL, "dst is NULL");
    const AdjWork a = adjoint_work(h, work);
    KParams kp = h->base;
    adjoint_params(h, kp, a, h->adj_cur, -1);
    h->ks->adj_copy(kp, h->L.nslots, h->L.nodes, dst, false, static_cast<hipStream_t>(stream));
    return launched("adjoint copy kernel");
}

int lbm_adjoint_set(lbm_handle* h, void* work, const double* src, void* stream) {
    if (int r = adjoint_ready(h, work)) return r;
    if (!src) return fail(LBM_EINVAL, "src is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const AdjWork a = adjoint_work(h, work);
    zero_partials(a, s);
    KParams kp = h->base;
    adjoint_params(h, kp, a, -1, 0);
    h->ks->adj_copy(kp, h->L.nslots, h->L.nodes, const_cast<double*>(src), true, s);
    h->adj_cur = 0;
    return launched("adjoint copy kernel");
}

int64_t lbm_step_count(const lbm_handle* h) { return h ? h->steps : -1; }

void lbm_destroy(lbm_handle* h) { delete h; }

}  // extern "C"
