// HIP kernels of the coupled lattice-Boltzmann step for gfx950.
//
// One fused kernel per (lattice family, mode, storage precision, tile).  A
// work-group owns a TX x TY column of nodes and marches along z over `zc` planes.
// When the capillary force (or the free-energy diagnostic) needs grad phi and
// lap phi, phi of three consecutive planes, each with a one-node ring, is staged
// in LDS: the work-group computes phi of plane z+1 (its own nodes from registers
// kept for the next iteration, ring nodes from L2-resident neighbour
// populations), then updates plane z.  Populations live in two copies (read one,
// write the other), so ring reads never race with writes.  Streaming is a pull:
// a copy holds post-collision populations; each node gathers X_k from x - e_k
// (periodic wrap), collides, and writes its post-collision populations to its
// own slots, so every store is aligned.  Half-way bounce-back at the z walls (the
// kernel frame's marching axis; the user's y axis in 2D) is taken when pulling: after
// a step a copy holds each node's raw post-collision populations, and a population
// X_k(x) whose source x - e_k lies beyond a z wall is read from the node's own slot
// opp(k) instead (zbounce).  Every reader of a state (step, moments, initialisation,
// population access, adjoint) follows this rule.  Walls on x and y are a small fix-up
// kernel after the step (k_walls).
//
// Memory layout of one copy: a sequence of slots, one [node] array per
// (field, direction) in the canonical order f_0.., g_0.., hA_0.., hB_0...  Every
// slot base is wave-uniform (SGPR) and every access uses a 32-bit per-lane
// offset, so each load / store is one `global_* voffset, saddr` instruction.
#pragma once

#include <cstddef>
#include <type_traits>

#include "adjoint.hpp"
#include "lattice.hpp"
#include "params.hpp"
#include "physics.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// helpers



// 1/x: exact in FP64, the hardware reciprocal (1 ulp) in FP32
template <class C>
__device__ __forceinline__ C rcp(C x) {
    if constexpr (std::is_same<C, double>::value) return 1.0 / x;
    else return __builtin_amdgcn_rcpf(x);
}

// Work-groups are handed to the 8 XCDs of the chip round-robin by linear id.
// Remap so that XCD j owns the contiguous range of tiles [j N / 8, (j + 1) N / 8):
// tiles that share phi-halo cache lines then run on the same XCD and meet in
// its L2 instead of each fetching the lines from memory.
__device__ __forceinline__ int xcd_tile(int w, int n) {
    constexpr int kXcd = 8;
    const int base = n / kXcd, rem = n % kXcd;
    const int j = w % kXcd, local = w / kXcd;
    return j < rem ? j * (base + 1) + local : rem * (base + 1) + (j - rem) * base + local;
}

// periodic wrap / mirror ghost of a coordinate in [-1, n]
__device__ __forceinline__ int map_coord(int c, int n, int wall) {
    if (c < 0) return wall ? 0 : n - 1;
    if (c >= n) return wall ? n - 1 : 0;
    return c;
}

// index offsets of the six axis neighbours of node (x, y, z), periodic wrap folded in
struct Nbr {
    int xp, xm, yp, ym, zp, zm;
};

__device__ __forceinline__ Nbr neighbours(int x, int y, int z, const KParams& P) {
    const int nxny = P.nx * P.ny;
    Nbr n;
    n.xp = (x + 1 < P.nx) ? 1 : 1 - P.nx;
    n.xm = (x > 0) ? -1 : P.nx - 1;
    n.yp = (y + 1 < P.ny) ? P.nx : (1 - P.ny) * P.nx;
    n.ym = (y > 0) ? -P.nx : (P.ny - 1) * P.nx;
    n.zp = (z + 1 < P.nz) ? nxny : (1 - P.nz) * nxny;
    n.zm = (z > 0) ? -nxny : (P.nz - 1) * nxny;
    return n;
}

// offset of the node x - e that a population moving along e arrives from (pull)
template <int EX, int EY, int EZ>
__device__ __forceinline__ int pull_offset(const Nbr& n) {
    int d = 0;
    if constexpr (EX > 0) d += n.xm;
    if constexpr (EX < 0) d += n.xp;
    if constexpr (EY > 0) d += n.ym;
    if constexpr (EY < 0) d += n.yp;
    if constexpr (EZ > 0) d += n.zm;
    if constexpr (EZ < 0) d += n.zp;
    return d;
}

// A 32-bit byte offset the optimiser may not widen to 64 bits (an empty asm with a
// register operand, no instruction).  Base (SGPR) + this offset selects the
// `global_* voffset, saddr` form instead of a 64-bit per-lane address.
__device__ __forceinline__ unsigned voff(unsigned byte_offset) {
    asm("" : "+v"(byte_offset));
    return byte_offset;
}

// index offsets of the axis neighbours for the phi stencil: periodic wrap, or the
// node itself beyond a wall (mirror ghost of a half-way wall)
__device__ __forceinline__ Nbr stencil_neighbours(int x, int y, int z, const KParams& P) {
    const int nxny = P.nx * P.ny;
    Nbr n;
    n.xp = (x + 1 < P.nx) ? 1 : (P.wall_x ? 0 : 1 - P.nx);
    n.xm = (x > 0) ? -1 : (P.wall_x ? 0 : P.nx - 1);
    n.yp = (y + 1 < P.ny) ? P.nx : (P.wall_y ? 0 : (1 - P.ny) * P.nx);
    n.ym = (y > 0) ? -P.nx : (P.wall_y ? 0 : (P.ny - 1) * P.nx);
    n.zp = (z + 1 < P.nz) ? nxny : (P.wall_z ? 0 : (1 - P.nz) * nxny);
    n.zm = (z > 0) ? -nxny : (P.wall_z ? 0 : (P.nz - 1) * nxny);
    return n;
}

// offset of the node x + e
template <int EX, int EY, int EZ>
__device__ __forceinline__ int push_offset(const Nbr& n) {
    return pull_offset<-EX, -EY, -EZ>(n);
}

// does the pull of a population moving along z-component EZ at a node on the low
// (zlo) or high (zhi) z wall plane cross the wall?  Then it bounces back: the node's
// own population of the opposite direction (Section 4.2.4, half-way bounce-back).
template <int EZ>
__device__ __forceinline__ bool zbounce(bool zlo, bool zhi) {
    if constexpr (EZ > 0) return zlo;
    else if constexpr (EZ < 0) return zhi;
    else return false;
}

// ---------------------------------------------------------------------------
// population storage

// slot bookkeeping of one lattice family: f, g, then NC composition fields (hA, hB,
// and hC with three compositions); rest slots (k = 0) are f_0, g_0, hA_0, hB_0 (, hC_0)
template <int QF, int QS, int NC = 2>
struct Slots {
    static constexpr int G0 = QF, A0 = QF + QS, B0 = QF + 2 * QS, C0 = QF + 3 * QS, N = QF + (1 + NC) * QS;
    __host__ __device__ static constexpr bool rest(int s) {
        return (QF > 0 && s == 0) || s == G0 || s == A0 || s == B0 || (NC >= 3 && s == C0);
    }
    __host__ __device__ static constexpr int rest_before(int s) {
        return (QF > 0 && s > 0 ? 1 : 0) + (s > G0 ? 1 : 0) + (s > A0 ? 1 : 0) + (s > B0 ? 1 : 0) +
               (NC >= 3 && s > C0 ? 1 : 0);
    }
    __host__ __device__ static constexpr int field(int s) {
        return s < G0 ? 0 : (s < A0 ? 1 : (s < B0 ? 2 : (s < C0 ? 3 : 4)));
    }
};

// byte offset of slot S in a copy (moving slots take stride_m bytes, rest slots stride_r)
template <class SLOTS, int S>
__device__ __forceinline__ unsigned long long slot_offset(const KParams& P) {
    constexpr int rb = SLOTS::rest_before(S);
    return (unsigned long long)(S - rb) * P.stride_m + (unsigned long long)rb * P.stride_r;
}

// where a reader finds X_k(x) (slot S = direction k of lattice L of a field): slot S at
// the pull source x - e_k, or the node's own slot of opp(k) when that crosses a z wall
// (zbounce).  Returns the slot base in `base`'s copy and the node index in t.
template <class SLOTS, class L, int S, int K>
__device__ __forceinline__ const char* pull_src(const char* base, const KParams& P, int z, unsigned idx,
                                                const Nbr& nb, unsigned& t) {
    if (zbounce<L::ez(K)>(P.wall_z && z == 0, P.wall_z && z == P.nz - 1)) {
        t = idx;
        return base + slot_offset<SLOTS, S - K + L::opp(K)>(P);
    }
    t = unsigned(int(idx) + pull_offset<L::ex(K), L::ey(K), L::ez(K)>(nb));
    return base + slot_offset<SLOTS, S>(P);
}

// load one population at node idx and decode it to the compute type
// NT: a non-temporal load, for data no other work-group reads
template <class T, bool NT>
__device__ __forceinline__ T ld_raw(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int PREC, bool REST, bool NT = false>
__device__ __forceinline__ typename Stor<PREC>::C ld_at(const char* slot, unsigned idx, float wref,
                                                        float inv_scale) {
    if constexpr (PREC == P64) {
        return ld_raw<double, NT>(reinterpret_cast<const double*>(slot + idx * 8u));
    } else if constexpr (PREC == P32 || REST) {
        return ld_raw<float, NT>(reinterpret_cast<const float*>(slot + idx * 4u));
    } else {
        const unsigned short bits = ld_raw<unsigned short, NT>(reinterpret_cast<const unsigned short*>(slot + idx * 2u));
        if constexpr (PREC == P16) return fmaf(__half2float(__ushort_as_half(bits)), inv_scale, wref);
        else return float(__builtin_bit_cast(__bf16, bits)) + wref;  // BF16: no scale
    }
}

// decode the low / high 16 bits of a word as a moving 16-bit population (the words of
// the packed LDS ring); the same arithmetic as ld_at
template <int PREC>
__device__ __forceinline__ float dec_lo(unsigned w, float wref, float inv_scale) {
    if constexpr (PREC == P16) return fmaf(__half2float(__ushort_as_half((unsigned short)(w & 0xffffu))), inv_scale, wref);
    else return __builtin_bit_cast(float, w << 16) + wref;
}
template <int PREC>
__device__ __forceinline__ float dec_hi(unsigned w, float wref, float inv_scale) {
    if constexpr (PREC == P16) return fmaf(__half2float(__ushort_as_half((unsigned short)(w >> 16))), inv_scale, wref);
    else return __builtin_bit_cast(float, w & 0xffff0000u) + wref;
}

// 16-bit encoding of one moving population: d = (v - w_k ref) 2^s in FP16, or v - w_k ref
// in BF16 (its exponent range is FP32's, so it takes no scale), rounded to nearest even
template <int PREC>
__device__ __forceinline__ float enc_d(float v, float wref, float scale) {
    if constexpr (PREC == P16) return (v - wref) * scale;
    else return v - wref;
}

// encode and store one population; populations written by a step are read again
// only in the next step, so they stream past the caches (non-temporal stores)
template <int PREC, bool REST>
__device__ __forceinline__ void st_at(char* slot, unsigned idx, float wref, float scale,
                                      typename Stor<PREC>::C v) {
    if constexpr (PREC == P64) {
        __builtin_nontemporal_store(v, reinterpret_cast<double*>(slot + idx * 8u));
    } else if constexpr (PREC == P32 || REST) {
        __builtin_nontemporal_store(float(v), reinterpret_cast<float*>(slot + idx * 4u));
    } else {
        const float d = enc_d<PREC>(v, wref, scale);
        unsigned short bits;
        if constexpr (PREC == P16) bits = __half_as_ushort(__float2half_rn(d));
        else bits = __builtin_bit_cast(unsigned short, __bf16(d));  // round to nearest even
        __builtin_nontemporal_store(bits, reinterpret_cast<unsigned short*>(slot + idx * 2u));
    }
}

// store, returning the value the slot now decodes to (16-bit moving populations:
// the rounded value; otherwise v itself)
template <int PREC, bool REST>
__device__ __forceinline__ typename Stor<PREC>::C st_at_r(char* slot, unsigned idx, float wref, float scale,
                                                           float inv_scale, typename Stor<PREC>::C v) {
    if constexpr (PREC == P64 || PREC == P32 || REST) {
        st_at<PREC, REST>(slot, idx, wref, scale, v);
        return v;
    } else {
        const float d = enc_d<PREC>(v, wref, scale);
        unsigned short bits;
        float back;
        if constexpr (PREC == P16) {
            const __half hd = __float2half_rn(d);
            bits = __half_as_ushort(hd);
            back = __half2float(hd) * inv_scale;
        } else {
            const __bf16 bd = __bf16(d);  // round to nearest even
            bits = __builtin_bit_cast(unsigned short, bd);
            back = float(bd);
        }
        __builtin_nontemporal_store(bits, reinterpret_cast<unsigned short*>(slot + idx * 2u));
        return back + wref;
    }
}

// store a moving 16-bit population and return its rounding residue in the encoded
// domain, d - round(d); (value - stored value) is that times 2^-s (FP16) or itself (BF16)
template <int PREC>
__device__ __forceinline__ float st_at_res(char* slot, unsigned idx, float wref, float scale, float v) {
    static_assert(PREC == P16 || PREC == PB16, "16-bit formats only");
    const float d = enc_d<PREC>(v, wref, scale);
    unsigned short bits;
    float back;
    if constexpr (PREC == P16) {
        const __half hd = __float2half_rn(d);
        bits = __half_as_ushort(hd);
        back = __half2float(hd);
    } else {
        const __bf16 bd = __bf16(d);  // round to nearest even
        bits = __builtin_bit_cast(unsigned short, bd);
        back = float(bd);
    }
    __builtin_nontemporal_store(bits, reinterpret_cast<unsigned short*>(slot + idx * 2u));
    return d - back;
}

// store two moving 16-bit populations of one field (slots sa, sb at node idx, the same
// reference w_k ref) with one packed conversion (round to nearest even); returns the sum
// of their stored deviations in the encoded domain
template <int PREC>
__device__ __forceinline__ float st2_at_dev(char* sa, char* sb, unsigned idx, float wref, float scale, float va,
                                            float vb) {
    static_assert(PREC == P16 || PREC == PB16, "16-bit formats only");
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 d = {enc_d<PREC>(va, wref, scale), enc_d<PREC>(vb, wref, scale)};
    unsigned bits;
    float back;
    if constexpr (PREC == P16) {
        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
        const h2 r = __builtin_convertvector(d, h2);
        bits = __builtin_bit_cast(unsigned, r);
        back = float(r.x) + float(r.y);
    } else {
        typedef __bf16 b2 __attribute__((ext_vector_type(2)));
        bits = __builtin_bit_cast(unsigned, __builtin_convertvector(d, b2));
        back = __builtin_bit_cast(float, bits << 16) + __builtin_bit_cast(float, bits & 0xffff0000u);
    }
    __builtin_nontemporal_store((unsigned short)(bits & 0xffffu), reinterpret_cast<unsigned short*>(sa + idx * 2u));
    __builtin_nontemporal_store((unsigned short)(bits >> 16), reinterpret_cast<unsigned short*>(sb + idx * 2u));
    return back;
}

// runtime-slot variants (generic copy kernels)
template <int PREC>
__device__ __forceinline__ typename Stor<PREC>::C ld_pop(const void* base, int idx, bool rest,
                                                         float wref, float inv_scale) {
    const char* p = static_cast<const char*>(base);
    if (rest) return ld_at<PREC, true>(p, unsigned(idx), wref, inv_scale);
    return ld_at<PREC, false>(p, unsigned(idx), wref, inv_scale);
}

template <int PREC>
__device__ __forceinline__ void st_pop(void* base, int idx, bool rest, float wref, float scale,
                                       typename Stor<PREC>::C v) {
    char* p = static_cast<char*>(base);
    if (rest) st_at<PREC, true>(p, unsigned(idx), wref, scale, v);
    else st_at<PREC, false>(p, unsigned(idx), wref, scale, v);
}

// ---------------------------------------------------------------------------
// block reduction of N doubles (entry `maxslot` takes a max, the others a sum),
// fixed order, one result per work-group

// ACC: add to out (each work-group owns its out entries, so repeated launches
// accumulate deterministically)
template <int N, int NT, bool ACC = false>
__device__ __forceinline__ void block_reduce_store(double (&v)[N], int maxslot, double* out) {
    static_assert(NT % 64 == 0, "work-group must be whole waves");
    __shared__ double red[NT / 64][N];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double o = __shfl_down(v[i], off, 64);
            v[i] = (i == maxslot) ? fmax(v[i], o) : v[i] + o;
        }
    }
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    if ((tid & 63) == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) red[tid >> 6][i] = v[i];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double a = red[0][i];
            for (int w = 1; w < NT / 64; ++w) a = (i == maxslot) ? fmax(a, red[w][i]) : a + red[w][i];
            if constexpr (ACC) out[i] += a;
            else out[i] = a;
        }
    }
}

// ---------------------------------------------------------------------------
// the fused step / moments / diagnostics kernel

#ifndef LBM_WAVES_PER_EU
#define LBM_WAVES_PER_EU 1
#endif
// occupancy target of the adjoint node kernel (register budget 512 / waves): the
// largest at which it does not spill (2D: 165 VGPRs, 3D: 234 VGPRs in FP32)
#ifndef LBM_ADJ_WAVES_2D
#define LBM_ADJ_WAVES_2D 3
#endif
#ifndef LBM_ADJ_WAVES_3D
#define LBM_ADJ_WAVES_3D 2
#endif
#ifndef LBM_EARLY_F
#define LBM_EARLY_F 1
#endif
#ifndef LBM_LDS_POPS
#define LBM_LDS_POPS 1
#endif
#ifndef LBM_NT_FLUID
#define LBM_NT_FLUID 1
#endif
#ifndef LBM_PHASES
#define LBM_PHASES 0
#endif
#ifndef LBM_FLAT_FILL
#define LBM_FLAT_FILL 1
#endif
#ifndef LBM_FRAW
#define LBM_FRAW 1
#endif

// scheduling fence between phases of the collision (bounds register live ranges)
#define LBM_FENCE()                                          \
    do {                                                     \
        if constexpr (LBM_PHASES) __builtin_amdgcn_sched_barrier(0); \
    } while (0)

// index of the pair (k, opp(k)), k < opp(k), among the moving directions of lattice L
template <class L, int K>
constexpr int pair_index() {
    int n = 0;
    for (int j = 1; j < K; ++j)
        if (j < L::opp(j)) ++n;
    return n;
}

// MRT relaxation of one field (the multiple-relaxation-time alternative to BGK):
// n_k = X_k - eqs(k) to the moment basis, moment i times rate(i) / <M_i, M_i>, back
// with M^-1_{k i} = w_k M_ik / <M_i, M_i>, then out(k, X_k - w_k (M^T m)_k + src(k)).
template <class L>
inline constexpr MomentBasis<L::Q> kBasis = make_moment_basis<L>();

template <class L, class C, class EQ, class SRC, class RATE, class OUT>
__device__ __forceinline__ void mrt_relax(const C (&X)[L::Q], EQ&& eqs, SRC&& src, RATE&& rate, OUT&& out) {
    constexpr int Q = L::Q;
    C n[Q], m[Q];
    static_for<0, Q>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        n[k] = X[k] - eqs(kc);
    });
    static_for<0, Q>([&](auto ic) __attribute__((always_inline)) {
        constexpr int i = decltype(ic)::value;
        C a = C(0);
        static_for<0, Q>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            constexpr double mik = kBasis<L>.M[i][k];
            if constexpr (mik != 0.0) a += C(mik) * n[k];
        });
        m[i] = a * (rate(ic) * C(kBasis<L>.invD[i]));
    });
    static_for<0, Q>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        C a = C(0);
        static_for<0, Q>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = decltype(ic)::value;
            constexpr double mik = kBasis<L>.M[i][k];
            if constexpr (mik != 0.0) a += C(mik) * m[i];
        });
        out(kc, X[k] - C(L::w(k)) * a + src(kc));
    });
}

// order of row i of the basis, and whether it is the trace of the second order
template <class L, int I>
constexpr int basis_order() { return kBasis<L>.order[I]; }
template <class L, int I>
constexpr bool basis_trace() { return kBasis<L>.order[I] == 2 && (I == 0 || kBasis<L>.order[I - 1] != 2); }

// occupancy floor of the fused kernel: one wave per SIMD (the compiler may use every
// register), except where a higher floor measured faster at 256^3:
// - the D3Q19 scalar lattices with 16-bit storage (the paper's 3D discretisation) and
//   the BGK, TRT or variable-density collisions, or MRT with BF16: with the packed LDS
//   ring they need about 260 registers; two waves per SIMD (256, at most 64 bytes of
//   spill) are 6-15 % faster than one;
// - D3Q7 with 16-bit storage, whose 3D launch puts three work-groups on a compute unit:
//   where the kernel needs more than 168 registers only two fit, and the 768 work-groups
//   of the 256^3 box run as one and a half rounds.  Three waves per SIMD (168 registers,
//   8-20 bytes of spill): general curvatures +27 % (BF16) and +8 % (FP16); a third
//   composition with BF16 (175 registers) +8 %.
// - 2D with 16-bit storage and flow, kernels of 129-146 registers (three waves): four
//   waves per SIMD measured at 2048^2 +9-13 % with a third composition, +13-14 % for the
//   variable-density model on D2Q9 scalars, +14 % for the paper's D2Q9 lattices with
//   FP16, +8 % for MRT on D2Q5 with BF16.
// Measured slower with the higher floor: MRT on D3Q7 (-16 %, 200 registers) and on D3Q19
// with FP16, the third composition on D3Q7 with FP16, the general-curvature D3Q19 and
// D2Q9 (FP16) kernels, the variable-density model on D2Q5 (BF16), and every kernel in
// FP32 / FP64
template <class SL, int PREC, int COLL, int NC = 2, int QF = 0>
constexpr int lbm_waves() {
    constexpr bool s16 = PREC == P16 || PREC == PB16;
    constexpr bool coll = (COLL & COLL_GK) == 0 && ((COLL & COLL_MRT) == 0 || PREC == PB16);
    if constexpr (s16 && SL::Q == 19 && coll) return 2;
    if constexpr (s16 && SL::Q == 7 && (COLL & COLL_GK) != 0) return 3;
    if constexpr (PREC == PB16 && SL::Q == 7 && NC == 3) return 3;
    if constexpr (s16 && SL::DIM == 2 && QF > 0) {
        if constexpr (NC == 3) return 4;
        if constexpr (SL::Q == 9 && COLL == COLL_VD) return 4;
        if constexpr (SL::Q == 9 && COLL == COLL_BGK && PREC == P16) return 4;
        if constexpr (SL::Q == 5 && COLL == COLL_MRT && PREC == PB16) return 4;
    }
    return LBM_WAVES_PER_EU;
}

template <class SL, class FL, int MODE, int PREC, int TX, int TY, int COLL = COLL_BGK, int NC = 2>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(lbm_waves<SL, PREC, COLL, NC, FL::Q>())))
k_lbm(const KParams P) {
    using C = typename Stor<PREC>::C;
    using SLOTS = Slots<FL::Q, SL::Q, NC>;
    constexpr int QS = SL::Q;
    constexpr int QF = FL::Q;
    constexpr bool FLOW = QF > 0;
    constexpr bool STENCIL = FLOW || MODE == MODE_DIAG;
    constexpr bool HAS_Y = SL::DIM == 3;
    using STL = typename std::conditional<SL::DIM == 2, D2Q9K, D3Q19K>::type;
    constexpr int LX = TX + 2;
    constexpr int LY = HAS_Y ? TY + 2 : 1;
    constexpr int OY = HAS_Y ? 1 : 0;
    constexpr int NSLOT = STENCIL ? 3 : 1;
    constexpr int NT = TX * TY;
    constexpr int G0 = SLOTS::G0, A0 = SLOTS::A0, B0 = SLOTS::B0, HC0 = SLOTS::C0;
    // NC = 3: a third independent composition C (N components), BGK Boussinesq step
    constexpr bool NC3 = NC == 3;
    constexpr int QC = NC3 ? QS : 1;
    static_assert(NC == 2 || (NC == 3 && COLL == COLL_BGK), "a third composition runs with the BGK Boussinesq step");
    static_assert(SLOTS::N <= kMaxSlots, "slot table too small for this lattice family");
    constexpr C inv_cs2s = C(1.0 / SL::cs2);
    constexpr bool TRTC = (COLL & COLL_TRT) != 0;
    constexpr bool MRTC = (COLL & COLL_MRT) != 0;
    constexpr bool VD = FLOW && (COLL & COLL_VD) != 0;
    constexpr bool GK = (COLL & COLL_GK) != 0;
    static_assert(TY == 1 || HAS_Y, "2D problems use one row per work-group");
    // the private LDS ring of scalar populations, unless it would not leave room for a
    // second work-group per compute unit (the paper's D3Q19 scalar lattice in FP32 / FP64,
    // and with the general-curvature collision or MRT with FP16).  The other D3Q19
    // kernels with 16-bit storage take the packed ring (30 words per node and plane,
    // 61 KB) and two waves per SIMD (lbm_waves)
    constexpr bool LDS_POPS = LBM_LDS_POPS && (lbm_waves<SL, PREC, COLL, NC, FL::Q>() == 2 ||
                                               2 * (1 + NC) * QS * NT * sizeof(C) <= 96 * 1024);
    static_assert((QS - 1) % 2 == 0, "moving directions come in opposite pairs");

    __shared__ C sphi[NSLOT][LY][LX];
    // this thread's own scalar populations of the current and the next plane
    // (thread-private ring of two planes, [plane][word][thread], no barriers needed).
    // FP32 / FP64: one word per population.  16-bit storage (PACKED): per field, the
    // FP32 rest population and the raw 16-bit moving populations of k and opp(k) packed
    // in one 32-bit word: 12 LDS words per node and plane instead of 21 (29 KB per
    // work-group instead of 48 KB; registers then bound the occupancy at three waves per
    // SIMD)
    constexpr bool PACKED = LDS_POPS && (PREC == P16 || PREC == PB16);
    constexpr int NPAIR = (QS - 1) / 2;
    constexpr int NWORD = PACKED ? (1 + NC) * (1 + NPAIR) : (1 + NC) * QS;
    using W = typename std::conditional<PACKED, unsigned, C>::type;
    __shared__ W spop[(STENCIL && LDS_POPS) ? 2 : 1][(STENCIL && LDS_POPS) ? NWORD : 1][(STENCIL && LDS_POPS) ? NT : 1];

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx;
    // tile of this work-group: x fastest, then y, then the z chunk
    const int tile = xcd_tile(blockIdx.x, P.tiles_x * P.tiles_y * P.tiles_z);
    const int bx = tile % P.tiles_x;
    const int by = (tile / P.tiles_x) % P.tiles_y;
    const int bz = tile / (P.tiles_x * P.tiles_y);
    const int x = bx * TX + tx;
    const int y = by * TY + ty;
    const bool active = (x < P.nx) && (y < P.ny);
    const int z0 = bz * P.zc;
    const int z1 = min(z0 + P.zc, P.nz);

    using SLT = std::common_type<SL>;  // type tags of the lattices
    using FLT = std::common_type<FL>;

    // wave-uniform slot bases of the source and destination copies.  The 2 x Q_tot
    // 64-bit bases do not fit in the SGPR file, and computing each from a copy base and
    // the slot strides costs about eight scalar instructions.  The host stores every
    // base in the parameter block; the kernel reads them through a kernel-argument
    // pointer that refresh_bases() makes opaque at the top of every plane, so each base
    // is one scalar load (merged with its neighbours) next to its use, and nothing is
    // hoisted into the SGPR file and spilled.
    using kconst = __attribute__((address_space(4))) const char;
    using kslot = __attribute__((address_space(4))) const unsigned long long;
    static_assert(offsetof(KParams, dst_slot) == offsetof(KParams, src_slot) + kMaxSlots * sizeof(void*),
                  "slot tables are adjacent");
    // the parameter block is the kernel's only argument, at offset 0 of the segment
    kconst* kargs = (kconst*)__builtin_amdgcn_kernarg_segment_ptr();
    auto refresh_bases = [&]() __attribute__((always_inline)) { asm volatile("" : "+s"(kargs)); };
    // the table entries lose the address space; the casts restore `global` so the
    // accesses stay global_* with a 32-bit voffset instead of flat_* with 64-bit addresses
    using gconst = __attribute__((address_space(1))) const char;
    using gmut = __attribute__((address_space(1))) char;
    auto src = [&](auto s_) __attribute__((always_inline)) -> const char* {
        constexpr int S = decltype(s_)::value;
        const unsigned long long b = reinterpret_cast<kslot*>(kargs + offsetof(KParams, src_slot))[S];
        return (const char*)(gconst*)b;
    };
    auto dst = [&](auto s_) __attribute__((always_inline)) -> char* {
        constexpr int S = decltype(s_)::value;
        const unsigned long long b = reinterpret_cast<kslot*>(kargs + offsetof(KParams, dst_slot))[S];
        return (char*)(gmut*)b;
    };
    // 16-bit reference w_k ref_field of slot S (direction k of lattice L): zero for the
    // compositions (their moving equilibria w_k mu are near zero) and for f in BF16 (its
    // deviations need no scale, and f ~ w_k p_h is centred on zero)
    constexpr bool NOREF_F = PREC == PB16;
    auto wref = [&](auto s_, auto k_, auto lat_) __attribute__((always_inline)) -> float {
        using L = typename decltype(lat_)::type;
        constexpr int F = SLOTS::field(decltype(s_)::value);
        if constexpr (F >= 2 || (F == 0 && NOREF_F)) return 0.0f;
        else return float(L::w(decltype(k_)::value)) * P.fref[F];
    };
    // the reference a decode adds: a zero reference as -0.0, since x + (-0.0) = x folds away
    // (x + 0.0 does not: it maps -0.0 to +0.0) and the encode's x - 0.0 folds as well
    auto wref_dec = [&](auto s_, auto k_, auto lat_) __attribute__((always_inline)) -> float {
        constexpr int F = SLOTS::field(decltype(s_)::value);
        if constexpr (F >= 2 || (F == 0 && NOREF_F)) return -0.0f;
        else return wref(s_, k_, lat_);
    };
    auto load = [&](auto s_, auto k_, auto lat_, unsigned idx) __attribute__((always_inline)) -> C {
        constexpr int S = decltype(s_)::value;
        return ld_at<PREC, SLOTS::rest(S)>(src(s_), idx, wref_dec(s_, k_, lat_), P.finv[SLOTS::field(S)]);
    };
    // fluid populations that arrive without an x shift are read by this work-group
    // only (no ring, no x neighbour shares their lines): streamed past the caches.
    // Measured: +1.7% for the 3D step, -1.7% for 2D (one row per work-group), so 3D only
    auto load_once = [&](auto s_, auto k_, auto lat_, unsigned idx) __attribute__((always_inline)) -> C {
        constexpr int S = decltype(s_)::value;
        using L = typename decltype(lat_)::type;
        constexpr bool NT = LBM_NT_FLUID && SL::DIM == 3 && L::ex(decltype(k_)::value) == 0;
        return ld_at<PREC, SLOTS::rest(S), NT>(src(s_), idx, wref_dec(s_, k_, lat_), P.finv[SLOTS::field(S)]);
    };
    auto store = [&](auto s_, auto k_, auto lat_, unsigned idx, C v) __attribute__((always_inline)) {
        constexpr int S = decltype(s_)::value;
        st_at<PREC, SLOTS::rest(S)>(dst(s_), idx, wref(s_, k_, lat_), P.fscale[SLOTS::field(S)], v);
    };
    // store a 16-bit moving population and add its rounding residue, in the encoded
    // domain, to res; fb<F>(res) is the residue in values of field F
    auto store_r = [&](auto s_, auto k_, auto lat_, unsigned idx, C v, C& res) __attribute__((always_inline)) {
        constexpr int S = decltype(s_)::value;
        static_assert(!SLOTS::rest(S), "rest populations carry no residue");
        res += st_at_res<PREC>(dst(s_), idx, wref(s_, k_, lat_), P.fscale[SLOTS::field(S)], v);
    };
    auto fb = [&](auto f_, C res) __attribute__((always_inline)) -> C {
        if constexpr (PREC == P16) return res * P.finv[decltype(f_)::value];
        else return res;
    };
    // sum of the stored moving populations of field F on lattice L, from the sum of their
    // stored deviations: sum_{k != 0} w_k ref_F + dev 2^-s
    auto stored_sum = [&](auto f_, auto lat_, C dev) __attribute__((always_inline)) -> C {
        using L = typename decltype(lat_)::type;
        constexpr int F = decltype(f_)::value;
        if constexpr (F >= 2 || (F == 0 && NOREF_F)) return fb(f_, dev);
        else return fb(f_, dev) + C(1.0 - L::w(0)) * P.fref[F];
    };

    // FP32 sum of the moving populations of one field, in the order k1, opp(k1), k2,
    // opp(k2), ... over k < opp(k) (16-bit storage; the packed LDS fill sums in this order)
    auto moving_sum = [&](const auto& x) __attribute__((always_inline)) -> C {
        C m = C(0);
        static_for<1, QS>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value, o = SL::opp(k);
            if constexpr (k < o) {
                if constexpr (pair_index<SL, k>() == 0) m = x[k] + x[o];
                else m = (m + x[k]) + x[o];
            }
        });
        return m;
    };

    // scalar populations arriving at node idx (pull from idx - e_k; the node's own
    // opposite population where that crosses a z wall: zlo / zhi, wave-uniform)
    // The scalar populations of a node in their stored form (RAW: 16-bit storage keeps
    // the bits of the moving populations and of the FP32 rest population, decoded later;
    // FP32 / FP64 the values), field-major: g, hA, hB (, hC), QS each
    constexpr bool RAW16 = PREC == P16 || PREC == PB16;
    constexpr int NSC = (1 + NC) * QS;
    using RW = typename std::conditional<RAW16, unsigned, C>::type;
    auto load_pops = [&](unsigned idx, const Nbr& nb, bool zlo, bool zhi, RW (&raw)[NSC]) __attribute__((always_inline)) {
        auto one = [&](auto s_, auto k_, unsigned t) __attribute__((always_inline)) -> RW {
            constexpr int S = decltype(s_)::value;
            if constexpr (!RAW16) return ld_at<PREC, SLOTS::rest(S)>(src(s_), t, 0.0f, 1.0f);
            else if constexpr (SLOTS::rest(S)) return __builtin_bit_cast(unsigned, ld_at<PREC, true>(src(s_), t, 0.0f, 1.0f));
            else return *reinterpret_cast<const unsigned short*>(src(s_) + t * 2u);
        };
        static_for<0, QS>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value, o = SL::opp(k);
            auto fields = [&](auto kk_, unsigned t) __attribute__((always_inline)) {
                constexpr int kk = decltype(kk_)::value;
                raw[k] = one(IC<G0 + kk>{}, kk_, t);
                raw[QS + k] = one(IC<A0 + kk>{}, kk_, t);
                raw[2 * QS + k] = one(IC<B0 + kk>{}, kk_, t);
                if constexpr (NC3) raw[3 * QS + k] = one(IC<HC0 + kk>{}, kk_, t);
            };
            if (zbounce<SL::ez(k)>(zlo, zhi)) fields(IC<o>{}, idx);
            else fields(kc, unsigned(int(idx) + pull_offset<SL::ex(k), SL::ey(k), SL::ez(k)>(nb)));
        });
    };
    // decoded values of one field (base slot B, first raw entry R0)
    auto decode_field = [&](auto b_, const RW* raw, C (&x)[QS]) __attribute__((always_inline)) {
        constexpr int B = decltype(b_)::value;
        static_for<0, QS>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            if constexpr (!RAW16) x[k] = raw[k];
            else if constexpr (k == 0) x[0] = __builtin_bit_cast(float, raw[0]);
            else x[k] = dec_lo<PREC>(raw[k], wref_dec(IC<B + k>{}, kc, SLT{}), P.finv[SLOTS::field(B)]);
        });
    };
    auto decode_pops = [&](const RW (&raw)[NSC], C (&gg)[QS], C (&aa)[QS], C (&bb)[QS], C (&qq)[QC])
                           __attribute__((always_inline)) {
        decode_field(IC<G0>{}, raw, gg);
        decode_field(IC<A0>{}, raw + QS, aa);
        decode_field(IC<B0>{}, raw + 2 * QS, bb);
        if constexpr (NC3) decode_field(IC<HC0>{}, raw + 3 * QS, qq);
    };
    auto pop_sums = [&](const C (&gg)[QS], const C (&aa)[QS], const C (&bb)[QS], const C (&qq)[QC], double& phis,
                        double& cA, double& cB, double& cC) __attribute__((always_inline)) {
        // zeroth moments.  mu = c - c^eq(phi) cancels c ~ 0.3 down to ~1e-3, so FP32
        // partial sums over all populations (several roundings of c and phi each) would
        // enter mu with a relative error near 1e-4 per step: FP32 / FP64 storage sums in
        // FP64.  16-bit storage sums its moving populations in FP32 and adds the FP32
        // rest population in FP64: the moving h are ~w_k mu (their FP32 sum is near
        // exact) and the moving g carry 16-bit storage noise far above FP32 rounding
        if constexpr (PREC == P16 || PREC == PB16) {
            phis = double(gg[0]) + double(moving_sum(gg));
            cA = double(aa[0]) + double(moving_sum(aa));
            cB = double(bb[0]) + double(moving_sum(bb));
            cC = NC3 ? double(qq[0]) + double(moving_sum(qq)) : 0.0;
        } else {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
            for (int k = 0; k < QS; ++k) {
                s0 += double(gg[k]);
                s1 += double(aa[k]);
                s2 += double(bb[k]);
                if constexpr (NC3) s3 += double(qq[k]);
            }
            phis = s0;
            cA = s1;
            cB = s2;
            cC = s3;
        }
    };
    auto load_scalars = [&](unsigned idx, const Nbr& nb, bool zlo, bool zhi, C (&gg)[QS], C (&aa)[QS],
                            C (&bb)[QS], C (&qq)[QC], double& phis, double& cA, double& cB, double& cC)
                            __attribute__((always_inline)) {
        RW raw[NSC];
        load_pops(idx, nb, zlo, zhi, raw);
        decode_pops(raw, gg, aa, bb, qq);
        pop_sums(gg, aa, bb, qq, phis, cA, cB, cC);
    };
    // phi of a node from its population sums (Eqs. Moment0_Phi, PotChem)
    auto phi_from = [&](double ps, double sa, double sb, double sc) __attribute__((always_inline)) -> double {
        if constexpr (NC3) return node_scalars3(ps, sa, sb, sc, P).phi;
        else return node_scalars<GK>(ps, sa, sb, P).phi;
    };

    auto node_phi = [&](int xx, int yy, int zz, bool zlo, bool zhi) __attribute__((always_inline)) -> C {
        C tg[QS], ta[QS], tb[QS], tq[QC];
        double ps, sa, sb, sc;
        load_scalars(unsigned((zz * P.ny + yy) * P.nx + xx), neighbours(xx, yy, zz, P), zlo, zhi, tg, ta, tb, tq,
                     ps, sa, sb, sc);
        return C(phi_from(ps, sa, sb, sc));
    };

    // scalar populations and sums of this thread's node: current plane (c*) and next plane (n*)
    C cg[QS], ca[QS], cb[QS], ng[QS], na[QS], nb[QS], cq[QC], nq[QC];
    double c_ps = 0.0, c_cA = 0.0, c_cB = 0.0, n_ps = 0.0, n_cA = 0.0, n_cB = 0.0, c_cC = 0.0, n_cC = 0.0;

    // phi of plane zz (tile + ring) into LDS slot `slot`; this thread's own node
    // populations go to the private LDS ring entry `pbuf` when the node is inside.
    // A z wall plane takes the bounce-back pulls (a separate, uniform branch: the
    // interior planes keep the plain loads)
    // PACKED: this node's own scalar populations (stored form) into the LDS ring (per
    // field: the FP32 rest population, then the moving populations of k and opp(k) in one
    // word) and their zeroth moments (the moving populations summed as moving_sum does)
    auto finish_packed = [&](const RW (&raw)[NSC], int pbuf, double& phis, double& cA, double& cB, double& cC)
                             __attribute__((always_inline)) {
      if constexpr (PACKED) {
        auto field = [&](auto b_, auto w0_, const RW* r, double& sum) __attribute__((always_inline)) {
            constexpr int B = decltype(b_)::value;    // slot of the field's rest population
            constexpr int W0 = decltype(w0_)::value;  // the field's first LDS word
            constexpr int F = SLOTS::field(B);
            spop[pbuf][W0][tid] = r[0];
            C m = C(0);
            static_for<1, QS>([&](auto kc) __attribute__((always_inline)) {
                constexpr int k = decltype(kc)::value, o = SL::opp(k);
                if constexpr (k < o) {
                    constexpr int PI = pair_index<SL, k>();
                    const unsigned w = r[k] | (r[o] << 16);
                    spop[pbuf][W0 + 1 + PI][tid] = w;
                    const C dk = dec_lo<PREC>(w, wref_dec(IC<B + k>{}, kc, SLT{}), P.finv[F]);
                    const C dd = dec_hi<PREC>(w, wref_dec(IC<B + o>{}, IC<o>{}, SLT{}), P.finv[F]);
                    if constexpr (PI == 0) m = dk + dd;
                    else m = (m + dk) + dd;
                }
            });
            sum = double(__builtin_bit_cast(float, r[0])) + double(m);
        };
        field(IC<G0>{}, IC<0>{}, raw, phis);
        field(IC<A0>{}, IC<1 + NPAIR>{}, raw + QS, cA);
        field(IC<B0>{}, IC<2 * (1 + NPAIR)>{}, raw + 2 * QS, cB);
        if constexpr (NC3) field(IC<HC0>{}, IC<3 * (1 + NPAIR)>{}, raw + 3 * QS, cC);
        else cC = 0.0;
      }
    };
    auto fill_packed = [&](unsigned idx, const Nbr& nb, bool zlo, bool zhi, int pbuf, double& phis, double& cA,
                           double& cB, double& cC) __attribute__((always_inline)) {
        RW raw[NSC];
        load_pops(idx, nb, zlo, zhi, raw);
        finish_packed(raw, pbuf, phis, cA, cB, cC);
    };

    // 3D plane fill with one memory round trip: every lane loads its own node (lanes
    // outside the domain an in-range stand-in) and one ring node (lanes beyond the ring
    // repeat its last node) in one basic block, so that all loads go out together; only
    // the waves that hold ring nodes decode them (a wave-uniform branch).  The stores
    // need no conditions: a lane's private LDS ring entries and the phi cells of lanes
    // outside the domain are never read, and a repeated ring node writes the same value
    // to the same cell.
    auto fill_body_flat = [&](int zm, bool zlo, bool zhi, int slot, int pbuf, double& ps, double& cA, double& cB,
                              double& cC) __attribute__((always_inline)) {
        constexpr int NH = 2 * LX + 2 * TY;
        static_assert(NT % 64 == 0, "whole waves");
        const int ox = map_coord(min(x, P.nx), P.nx, P.wall_x), oy = map_coord(min(y, P.ny), P.ny, P.wall_y);
        const int i = min(tid, NH - 1);
        int hx, hy;
        if (i < LX) { hx = i; hy = 0; }
        else if (i < 2 * LX) { hx = i - LX; hy = TY + 1; }
        else if (i < 2 * LX + TY) { hx = 0; hy = i - 2 * LX + 1; }
        else { hx = LX - 1; hy = i - 2 * LX - TY + 1; }
        const int rx = map_coord(min(bx * TX + hx - 1, P.nx), P.nx, P.wall_x);
        const int ry = map_coord(min(by * TY + hy - 1, P.ny), P.ny, P.wall_y);
        RW own[NSC], ring[NSC];
        load_pops(unsigned((zm * P.ny + oy) * P.nx + ox), neighbours(ox, oy, zm, P), zlo, zhi, own);
        load_pops(unsigned((zm * P.ny + ry) * P.nx + rx), neighbours(rx, ry, zm, P), zlo, zhi, ring);
        // keep the scheduler from moving the decode and sums of the own node between the
        // loads (it would then wait for them before the ring loads go out)
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (PACKED) {
            finish_packed(own, pbuf, ps, cA, cB, cC);
        } else if constexpr (LDS_POPS) {
            C gg[QS], aa[QS], bb[QS], qq[QC];
            decode_pops(own, gg, aa, bb, qq);
#pragma unroll
            for (int k = 0; k < QS; ++k) {
                spop[pbuf][k][tid] = gg[k];
                spop[pbuf][QS + k][tid] = aa[k];
                spop[pbuf][2 * QS + k][tid] = bb[k];
                if constexpr (NC3) spop[pbuf][3 * QS + k][tid] = qq[k];
            }
            pop_sums(gg, aa, bb, qq, ps, cA, cB, cC);
        } else {
            decode_pops(own, ng, na, nb, nq);
            pop_sums(ng, na, nb, nq, ps, cA, cB, cC);
        }
        sphi[slot][ty + OY][tx + 1] = C(phi_from(ps, cA, cB, cC));
        // the first lane of this wave holds a ring node (wave-uniform)
        if (__builtin_amdgcn_readfirstlane(tid) < NH) {
            C tg[QS], ta[QS], tb[QS], tq[QC];
            double rps, rsa, rsb, rsc;
            decode_pops(ring, tg, ta, tb, tq);
            pop_sums(tg, ta, tb, tq, rps, rsa, rsb, rsc);
            sphi[slot][hy][hx] = C(phi_from(rps, rsa, rsb, rsc));
        }
    };

    auto fill_body = [&](int zm, bool zlo, bool zhi, int slot, int pbuf, double& ps, double& cA, double& cB,
                         double& cC) __attribute__((always_inline)) {
        if constexpr (HAS_Y && LBM_FLAT_FILL) {
            fill_body_flat(zm, zlo, zhi, slot, pbuf, ps, cA, cB, cC);
            return;
        }
        if (active) {
            if constexpr (PACKED) {
                fill_packed(unsigned((zm * P.ny + y) * P.nx + x), neighbours(x, y, zm, P), zlo, zhi, pbuf, ps, cA, cB,
                            cC);
            } else if constexpr (LDS_POPS) {
                C gg[QS], aa[QS], bb[QS], qq[QC];
                load_scalars(unsigned((zm * P.ny + y) * P.nx + x), neighbours(x, y, zm, P), zlo, zhi, gg, aa, bb,
                             qq, ps, cA, cB, cC);
#pragma unroll
                for (int k = 0; k < QS; ++k) {
                    spop[pbuf][k][tid] = gg[k];
                    spop[pbuf][QS + k][tid] = aa[k];
                    spop[pbuf][2 * QS + k][tid] = bb[k];
                    if constexpr (NC3) spop[pbuf][3 * QS + k][tid] = qq[k];
                }
            } else {
                load_scalars(unsigned((zm * P.ny + y) * P.nx + x), neighbours(x, y, zm, P), zlo, zhi, ng, na, nb,
                             nq, ps, cA, cB, cC);
            }
            sphi[slot][ty + OY][tx + 1] = C(phi_from(ps, cA, cB, cC));
        } else if (x <= P.nx && y <= P.ny) {
            // ghost column / row just beyond the domain edge
            sphi[slot][ty + OY][tx + 1] = node_phi(map_coord(x, P.nx, P.wall_x),
                                                   HAS_Y ? map_coord(y, P.ny, P.wall_y) : 0, zm, zlo, zhi);
        }
        constexpr int NH = HAS_Y ? 2 * LX + 2 * TY : 2;
        for (int i = tid; i < NH; i += NT) {
            int hx, hy;
            if constexpr (HAS_Y) {
                if (i < LX) { hx = i; hy = 0; }
                else if (i < 2 * LX) { hx = i - LX; hy = TY + 1; }
                else if (i < 2 * LX + TY) { hx = 0; hy = i - 2 * LX + 1; }
                else { hx = LX - 1; hy = i - 2 * LX - TY + 1; }
            } else {
                hx = (i == 0) ? 0 : LX - 1;
                hy = 0;
            }
            const int gx = bx * TX + hx - 1;
            const int gy = HAS_Y ? by * TY + hy - 1 : 0;
            if (gx > P.nx || gy > P.ny) continue;  // beyond the ghost layer: never read
            sphi[slot][hy][hx] = node_phi(map_coord(gx, P.nx, P.wall_x),
                                          HAS_Y ? map_coord(gy, P.ny, P.wall_y) : 0, zm, zlo, zhi);
        }
    };
    auto fill_plane = [&](int zz, int slot, int pbuf, double& ps, double& cA, double& cB, double& cC)
                          __attribute__((always_inline)) {
        const int zm = map_coord(zz, P.nz, P.wall_z);
        const bool zlo = P.wall_z && zm == 0, zhi = P.wall_z && zm == P.nz - 1;
        if (zlo || zhi) fill_body(zm, zlo, zhi, slot, pbuf, ps, cA, cB, cC);
        else fill_body(zm, false, false, slot, pbuf, ps, cA, cB, cC);
    };

    // diagnostics: the kNumDiag reductions, then sum c^C with a third composition
    constexpr int NACC = (MODE == MODE_DIAG) ? (NC3 ? kNumDiag + 1 : kNumDiag) : 1;
    // this node's scalar populations of plane z from the private LDS ring into registers
    // (read right after the barrier: reading them only where the g and h collisions use
    // them frees about 18 VGPRs but measured 17 % slower, the LDS latency exposed)
    auto fetch_pops = [&](int zz) __attribute__((always_inline)) {
        if constexpr (PACKED && STENCIL) {
            if (active) {
                const int pb = (zz - z0) & 1;
                auto field = [&](auto b_, auto w0_, C(&x)[QS]) __attribute__((always_inline)) {
                    constexpr int B = decltype(b_)::value;
                    constexpr int W0 = decltype(w0_)::value;
                    constexpr int F = SLOTS::field(B);
                    x[0] = __builtin_bit_cast(float, spop[pb][W0][tid]);
                    static_for<1, QS>([&](auto kc) __attribute__((always_inline)) {
                        constexpr int k = decltype(kc)::value, o = SL::opp(k);
                        if constexpr (k < o) {
                            const unsigned w = spop[pb][W0 + 1 + pair_index<SL, k>()][tid];
                            x[k] = dec_lo<PREC>(w, wref_dec(IC<B + k>{}, kc, SLT{}), P.finv[F]);
                            x[o] = dec_hi<PREC>(w, wref_dec(IC<B + o>{}, IC<o>{}, SLT{}), P.finv[F]);
                        }
                    });
                };
                field(IC<G0>{}, IC<0>{}, cg);
                field(IC<A0>{}, IC<1 + NPAIR>{}, ca);
                field(IC<B0>{}, IC<2 * (1 + NPAIR)>{}, cb);
                if constexpr (NC3) field(IC<HC0>{}, IC<3 * (1 + NPAIR)>{}, cq);
            }
        } else if constexpr (LDS_POPS && STENCIL) {
            if (active) {
                const int pb = (zz - z0) & 1;
#pragma unroll
                for (int k = 0; k < QS; ++k) {
                    cg[k] = spop[pb][k][tid];
                    ca[k] = spop[pb][QS + k][tid];
                    cb[k] = spop[pb][2 * QS + k][tid];
                    if constexpr (NC3) cq[k] = spop[pb][3 * QS + k][tid];
                }
            }
        }
    };
    double acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = 0.0;

    const double phi_ref = P.mean_subtract ? *P.phi_ref : 0.0;
    // a model constant in the compute type (the FP32 copy for FP32 arithmetic)
    auto KC = [&](double d, float f) __attribute__((always_inline)) -> C {
        if constexpr (std::is_same<C, float>::value) return f;
        else return C(d);
    };
    if constexpr (MODE == MODE_STEP || MODE == MODE_STEP_PHI) {
        // a step between caller checkpoints carries the buffered <phi> over
        if (P.ref_copy && blockIdx.x == 0 && tid == 0) *P.ref_copy = *P.phi_ref;
    }

    if constexpr (STENCIL) {
        if (z0 < z1) {
            fill_plane(z0 - 1, 0, 1, n_ps, n_cA, n_cB, n_cC);  // ring only; own entries overwritten next
            fill_plane(z0, 1, 0, c_ps, c_cA, c_cB, c_cC);
            if constexpr (!LDS_POPS) {
#pragma unroll
                for (int k = 0; k < QS; ++k) { cg[k] = ng[k]; ca[k] = na[k]; cb[k] = nb[k]; }
                if constexpr (NC3) {
#pragma unroll
                    for (int k = 0; k < QS; ++k) cq[k] = nq[k];
                }
            }
        }
    }

    for (int z = z0; z < z1; ++z) {
        refresh_bases();
        int sm = 0, sc = 0, sp = 0;
        const unsigned idx = unsigned((z * P.ny + y) * P.nx + x);
        const Nbr nbr = neighbours(x, y, z, P);
        C fpop[QF > 0 ? QF : 1];
        // 16-bit storage: the moving f arrive as raw bits and are decoded where the flow
        // moments need them, so that no wait for them sits before the plane fill's loads
        constexpr bool FRAW = LBM_FRAW && (PREC == P16 || PREC == PB16);
        unsigned fraw[(QF > 0 && FRAW) ? QF : 1];
        auto load_f_body = [&](bool zlo, bool zhi) __attribute__((always_inline)) {
            static_for<0, QF>([&](auto kc) __attribute__((always_inline)) {
                constexpr int k = decltype(kc)::value, o = FL::opp(k);
                if constexpr (FRAW && k != 0) {
                    constexpr bool NT = LBM_NT_FLUID && SL::DIM == 3 && FL::ex(k) == 0;
                    const char* base;
                    unsigned t;
                    if (zbounce<FL::ez(k)>(zlo, zhi)) {
                        base = src(IC<o>{});
                        t = idx;
                    } else {
                        base = src(kc);
                        t = unsigned(int(idx) + pull_offset<FL::ex(k), FL::ey(k), FL::ez(k)>(nbr));
                    }
                    fraw[k] = ld_raw<unsigned short, NT>(reinterpret_cast<const unsigned short*>(base + t * 2u));
                } else if (zbounce<FL::ez(k)>(zlo, zhi)) {
                    fpop[k] = load_once(IC<o>{}, IC<o>{}, FLT{}, idx);
                } else {
                    const unsigned src_idx = unsigned(int(idx) + pull_offset<FL::ex(k), FL::ey(k), FL::ez(k)>(nbr));
                    fpop[k] = load_once(kc, kc, FLT{}, src_idx);
                }
            });
        };
        // 16-bit storage: z-wall bounce-back by selecting the source slot and node (no
        // branch: the loads stay in one basic block with the plane fill's)
        auto load_f_sel = [&]() __attribute__((always_inline)) {
            const bool zlo = P.wall_z && z == 0, zhi = P.wall_z && z == P.nz - 1;
            // lanes outside the domain load an in-range node (their values are not used)
            const int fx = min(x, P.nx - 1), fy = min(y, P.ny - 1);
            const unsigned fidx = unsigned((z * P.ny + fy) * P.nx + fx);
            const Nbr fnb = neighbours(fx, fy, z, P);
            static_for<0, QF>([&](auto kc) __attribute__((always_inline)) {
                constexpr int k = decltype(kc)::value, o = FL::opp(k);
                if constexpr (k != 0) {
                    constexpr bool NT = LBM_NT_FLUID && SL::DIM == 3 && FL::ex(k) == 0;
                    const unsigned pulled = unsigned(int(fidx) + pull_offset<FL::ex(k), FL::ey(k), FL::ez(k)>(fnb));
                    const char* base = src(kc);
                    unsigned t = pulled;
                    if constexpr (FL::ez(k) != 0) {
                        const bool b = zbounce<FL::ez(k)>(zlo, zhi);
                        base = b ? src(IC<o>{}) : base;
                        t = b ? fidx : pulled;
                    }
                    fraw[k] = ld_raw<unsigned short, NT>(reinterpret_cast<const unsigned short*>(base + t * 2u));
                } else {
                    fpop[0] = load_once(kc, kc, FLT{}, fidx);
                }
            });
        };
        auto load_f = [&]() __attribute__((always_inline)) {
            if constexpr (FLOW) {
                if constexpr (FRAW && HAS_Y && LBM_FLAT_FILL) {
                    load_f_sel();  // every lane loads (lanes outside the domain: in-range stand-ins)
                } else if (active) {
                    const bool zlo = P.wall_z && z == 0, zhi = P.wall_z && z == P.nz - 1;
                    if (zlo || zhi) load_f_body(zlo, zhi);
                    else load_f_body(false, false);
                }
            }
        };
        // fluid populations of this node do not depend on the LDS plane: with
        // LBM_EARLY_F they are issued before the plane fill to overlap its latency
        if constexpr (LBM_EARLY_F) load_f();
        if constexpr (STENCIL) {
            sm = (z - z0) % 3;
            sc = (z - z0 + 1) % 3;
            sp = (z - z0 + 2) % 3;
            fill_plane(z + 1, sp, (z - z0 + 1) & 1, n_ps, n_cA, n_cB, n_cC);
            __syncthreads();
            if constexpr (LDS_POPS) fetch_pops(z);
        } else {
            if (active) {
                const bool zlo = P.wall_z && z == 0, zhi = P.wall_z && z == P.nz - 1;
                if (zlo || zhi) load_scalars(idx, nbr, zlo, zhi, cg, ca, cb, cq, c_ps, c_cA, c_cB, c_cC);
                else load_scalars(idx, nbr, false, false, cg, ca, cb, cq, c_ps, c_cA, c_cB, c_cC);
            }
        }
        if constexpr (!LBM_EARLY_F) load_f();
        const C(&g)[QS] = cg;
        const C(&a)[QS] = ca;
        const C(&b)[QS] = cb;
        const double sA = c_cA, sB = c_cB, sC = c_cC;

        if (active) {
            Scalars m;
            double muC = 0.0;  // potential of a third composition
            if constexpr (NC3) {
                const Scalars3 m3 = node_scalars3(c_ps, sA, sB, sC, P);
                m = Scalars{m3.phi, m3.muA, m3.muB, m3.S};
                muC = m3.muC;
            } else {
                m = node_scalars<GK>(c_ps, sA, sB, P);
            }
            const C phi = C(m.phi);

            // isotropic gradient and Laplacian, Eqs. Grad and Laplacian (fluid lattice)
            C grad[3] = {C(0), C(0), C(0)};
            C lap = C(0);
            C pc = phi;
            C nsum = C(0);  // 3 sum_{k != 0} w_k phi(x + e_k)
            if constexpr (STENCIL) {
                pc = sphi[sc][ty + OY][tx + 1];
                static_for<1, STL::Q>([&](auto kc) __attribute__((always_inline)) {
                    constexpr int k = decltype(kc)::value;
                    constexpr int ex = STL::ex(k), ey = STL::ey(k), ez = STL::ez(k);
                    const int slot = ez == 0 ? sc : (ez > 0 ? sp : sm);
                    const C v = sphi[slot][ty + OY + ey][tx + 1 + ex];
                    const C wv = C(3.0 * STL::w(k)) * v;
                    if constexpr (ex != 0) grad[0] += ex > 0 ? wv : -wv;
                    if constexpr (ey != 0) grad[1] += ey > 0 ? wv : -wv;
                    if constexpr (ez != 0) grad[2] += ez > 0 ? wv : -wv;
                    nsum += wv;
                });
                lap = C(2) * (nsum - C(3.0 * (1.0 - STL::w(0))) * pc);
            }

            C u[3] = {C(0), C(0), C(0)};
            C p_h = C(0);  // pressure variable of f: p_h, or p* with variable density
            C F[3] = {C(0), C(0), C(0)};
            C irho = C(1);  // 1 / rho(phi) (variable density)
            if constexpr (FLOW) {
                // Eq. SurfaceTension_Force plus buoyancy (phi - phi_ref) drho g
                const C bracket = KC(P.cap, P.f32.cap) * (C(dwell_d(m.phi)) * KC(P.inv_W2, P.f32.inv_W2) - lap);
                const C buoy = C(m.phi - phi_ref) * KC(P.drho, P.f32.drho);
                F[0] = buoy * KC(P.gx, P.f32.gx) + bracket * grad[0];
                F[1] = buoy * KC(P.gy, P.f32.gy) + bracket * grad[1];
                F[2] = buoy * KC(P.gz, P.f32.gz) + bracket * grad[2];
                if constexpr (FRAW) {
                    static_for<1, QF>([&](auto kc) __attribute__((always_inline)) {
                        fpop[decltype(kc)::value] = dec_lo<PREC>(fraw[decltype(kc)::value], wref_dec(kc, kc, FLT{}), P.finv[0]);
                    });
                }
                // Eqs. HydroPressure and Velocity
                C j0 = C(0), j1 = C(0), j2 = C(0);
                static_for<0, QF>([&](auto kc) __attribute__((always_inline)) {
                    constexpr int k = decltype(kc)::value;
                    p_h += fpop[k];
                    if constexpr (FL::ex(k) != 0) j0 += FL::ex(k) > 0 ? fpop[k] : -fpop[k];
                    if constexpr (FL::ey(k) != 0) j1 += FL::ey(k) > 0 ? fpop[k] : -fpop[k];
                    if constexpr (FL::ez(k) != 0) j2 += FL::ez(k) > 0 ? fpop[k] : -fpop[k];
                });
                if constexpr (!VD) {
                    const C inv_rho0 = KC(1.0 / P.rho0, P.f32.inv_rho0);
                    u[0] = (C(3) * j0 + C(0.5) * F[0]) * inv_rho0;
                    u[1] = (C(3) * j1 + C(0.5) * F[1]) * inv_rho0;
                    u[2] = (C(3) * j2 + C(0.5) * F[2]) * inv_rho0;
                } else {
                    // variable density: f is dimensionless, p_h holds p* = sum f; rho(phi)
                    // interpolated; pressure force -p* c_s^2 grad rho; predictor velocity;
                    // viscous force -(nu w+ / c_s^2) Pi . grad rho from the non-equilibrium
                    // second moment at the predictor; final velocity
                    const C drho = KC(P.drho, P.f32.drho);
                    irho = rcp<C>(KC(P.rho0, P.f32.rho0) + drho * phi);
                    const C fp = -p_h * C(1.0 / 3.0) * drho;
                    C us[3];
                    us[0] = j0 + C(0.5) * (F[0] + fp * grad[0]) * irho;
                    us[1] = j1 + C(0.5) * (F[1] + fp * grad[1]) * irho;
                    us[2] = j2 + C(0.5) * (F[2] + fp * grad[2]) * irho;
                    const C uus = us[0] * us[0] + us[1] * us[1] + us[2] * us[2];
                    const C e0s = p_h - C(1.5) * uus;
                    C pxx = C(0), pyy = C(0), pzz = C(0), pxy = C(0), pxz = C(0), pyz = C(0);
                    static_for<0, QF>([&](auto kc) __attribute__((always_inline)) {
                        constexpr int k = decltype(kc)::value;
                        constexpr int ex = FL::ex(k), ey = FL::ey(k), ez = FL::ez(k);
                        const C eu = edot<ex, ey, ez>(us[0], us[1], us[2]);
                        const C n = fpop[k] - C(FL::w(k)) * (e0s + eu * (C(3) + C(4.5) * eu));
                        if constexpr (ex != 0) pxx += n;
                        if constexpr (ey != 0) pyy += n;
                        if constexpr (ez != 0) pzz += n;
                        if constexpr (ex != 0 && ey != 0) pxy += ex * ey > 0 ? n : -n;
                        if constexpr (ex != 0 && ez != 0) pxz += ex * ez > 0 ? n : -n;
                        if constexpr (ey != 0 && ez != 0) pyz += ey * ez > 0 ? n : -n;
                    });
                    const C nuv = KC(P.nu0, P.f32.nu0) * (C(1) - phi) + KC(P.nu1, P.f32.nu1) * phi;
                    const C coef = -C(3) * nuv * rcp<C>(C(3) * nuv + C(0.5)) * drho;
                    const C Fm[3] = {coef * (pxx * grad[0] + pxy * grad[1] + pxz * grad[2]),
                                     coef * (pxy * grad[0] + pyy * grad[1] + pyz * grad[2]),
                                     coef * (pxz * grad[0] + pyz * grad[1] + pzz * grad[2])};
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        u[a] = us[a] + C(0.5) * Fm[a] * irho;
                        F[a] += fp * grad[a] + Fm[a];
                    }
                }
            }

            if constexpr (MODE == MODE_STEP || MODE == MODE_STEP_PHI) {
                if (P.mean_subtract) acc[0] += m.phi;
                // phi of the source state, as the stencil saw it (for the adjoint)
                if constexpr (MODE == MODE_STEP_PHI) static_cast<C*>(P.phi_out)[idx] = phi;

                // post-collision populations go to this node's own slots of the other copy.
                // 16-bit storage: the rounding residue of a field's moving populations is
                // added to its FP32 rest population, so the stored state keeps each node's
                // post-collision mass of every field (the rest population is stored last)
                constexpr bool FEEDBACK = PREC == P16 || PREC == PB16;
                auto push = [&](auto s_, auto k_, auto lat_, C v) __attribute__((always_inline)) {
                    store(s_, k_, lat_, idx, v);
                };
                auto push_r = [&](auto s_, auto k_, auto lat_, C v, C& res) __attribute__((always_inline)) {
                    if constexpr (FEEDBACK) store_r(s_, k_, lat_, idx, v, res);
                    else store(s_, k_, lat_, idx, v);
                };
                // BGK steps: the moving populations of directions k and opp(k) of one field
                // (with 16-bit storage: one packed conversion; their stored deviations add to
                // dev, and the rest population is stored last as the field's post-collision
                // zeroth moment, conserved by the collision, minus the stored moving
                // populations, stored_sum)
                auto push_d2 = [&](auto sk_, auto so_, auto k_, auto o_, auto lat_, C vk, C vo, C& dev)
                                   __attribute__((always_inline)) {
                    if constexpr (FEEDBACK) {
                        constexpr int F = SLOTS::field(decltype(sk_)::value);
                        static_assert(F == SLOTS::field(decltype(so_)::value), "one field");
                        dev += st2_at_dev<PREC>(dst(sk_), dst(so_), idx, wref(sk_, k_, lat_), P.fscale[F], vk, vo);
                    } else {
                        store(sk_, k_, lat_, idx, vk);
                        store(so_, o_, lat_, idx, vo);
                    }
                };

                // ---- f: Eqs. LBE_FluidFlow, ForcingTerm, GammaFunction, Feq ----
                // f* = (1 - w) f + w w_k [p + rho0 (eu + 3/2 eu^2 - uu/2)] + (1 - w/2) F_k,
                // F_k = w_k [1 + 3 eu + 9/2 eu^2 - 3/2 uu] (e_k . F - u . F)
                if constexpr (FLOW) {
                    const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                    const C uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
                    const C nu = KC(P.nu0, P.f32.nu0) * (C(1) - phi) + KC(P.nu1, P.f32.nu1) * phi;
                    const C wf = rcp<C>(C(3) * nu + C(0.5));
                    const C keep = C(1) - wf, half = C(1) - C(0.5) * wf;
                    // inertia of the equilibrium: rho0 (Eq. Feq), or 1 / c_s^2 for the
                    // dimensionless populations of the variable-density model, whose
                    // forcing populations are divided by rho c_s^2
                    const C rho0 = VD ? C(3) : KC(P.rho0, P.f32.rho0);
                    const C g0 = C(1) - C(1.5) * uu, e0 = p_h - C(0.5) * rho0 * uu;
                    const C fsc = VD ? C(3) * irho : C(1);
                    if constexpr (MRTC) {
                        // MRT: the traceless second order at the viscous rate wf, the trace,
                        // third and fourth orders at the given rates; orders 0 and 1 are
                        // conserved (rate 1)
                        auto feqs = [&](auto kc, C& Fk) __attribute__((always_inline)) -> C {
                            constexpr int k = decltype(kc)::value;
                            constexpr int ex = FL::ex(k), ey = FL::ey(k), ez = FL::ez(k);
                            const C wk = C(FL::w(k));
                            const C eu = edot<ex, ey, ez>(u[0], u[1], u[2]);
                            const C eF = edot<ex, ey, ez>(F[0], F[1], F[2]);
                            Fk = wk * (g0 + eu * (C(3) + C(4.5) * eu)) * (eF - uF);
                            if constexpr (VD) Fk *= fsc;
                            return wk * (e0 + rho0 * eu * (C(1) + C(1.5) * eu)) - C(0.5) * Fk;
                        };
                        C Fks[QF];
                        C resm = C(0), restm = C(0);
                        mrt_relax<FL>(fpop,
                            [&](auto kc) __attribute__((always_inline)) -> C {
                                return feqs(kc, Fks[decltype(kc)::value]);
                            },
                            [&](auto kc) __attribute__((always_inline)) -> C { return Fks[decltype(kc)::value]; },
                            [&](auto ic) __attribute__((always_inline)) -> C {
                                constexpr int i = decltype(ic)::value;
                                constexpr int o = basis_order<FL, i>();
                                if constexpr (o <= 1) return C(1);
                                else if constexpr (basis_trace<FL, i>()) return KC(P.mrt_f[0], P.f32.mrt_f[0]);
                                else if constexpr (o == 2) return wf;
                                else if constexpr (o == 3) return KC(P.mrt_f[1], P.f32.mrt_f[1]);
                                else return KC(P.mrt_f[2], P.f32.mrt_f[2]);
                            },
                            [&](auto kc, C v) __attribute__((always_inline)) {
                                if constexpr (decltype(kc)::value == 0 && FEEDBACK) restm = v;
                                else push_r(kc, kc, FLT{}, v, resm);
                            });
                        if constexpr (FEEDBACK) push(IC<0>{}, IC<0>{}, FLT{}, restm + fb(IC<0>{}, resm));
                    } else if constexpr (!TRTC) {
                    // f*_k = keep f_k + w_k [a_k + gam_k (e_k . Fh - u . Fh)] with
                    // a_k = wf (e0 + rho0 (eu + 3/2 eu^2)), gam_k = 1 + 3 eu + 9/2 eu^2 - 3/2 uu
                    // and Fh = (1 - wf/2) F (times 1 / (rho c_s^2) with variable density):
                    // k and opp(k) share eu^2 and differ in the signs of eu, e_k . Fh
                    const C A = wf * e0, B = wf * rho0;
                    const C hs = half * fsc;
                    const C Fh[3] = {hs * F[0], hs * F[1], hs * F[2]};
                    const C uFh = hs * uF;
                    C dev = C(0);
                    static_for<1, QF>([&](auto kc) __attribute__((always_inline)) {
                        constexpr int k = decltype(kc)::value;
                        constexpr int o = FL::opp(k);
                        if constexpr (k < o) {
                            constexpr int ex = FL::ex(k), ey = FL::ey(k), ez = FL::ez(k);
                            const C wk = C(FL::w(k));  // w_opp(k) = w_k
                            const C eu = edot<ex, ey, ez>(u[0], u[1], u[2]);
                            const C eF = edot<ex, ey, ez>(Fh[0], Fh[1], Fh[2]);
                            const C e2 = eu * eu;
                            const C q = C(1.5) * e2;
                            const C r = g0 + C(4.5) * e2;
                            const C ak = A + B * (q + eu), ao = A + B * (q - eu);
                            const C gk = r + C(3) * eu, go = r - C(3) * eu;
                            const C vk = keep * fpop[k] + wk * (ak + gk * (eF - uFh));
                            const C vo = keep * fpop[o] + wk * (ao - go * (eF + uFh));
                            push_d2(kc, IC<o>{}, kc, IC<o>{}, FLT{}, vk, vo, dev);
                        }
                    });
                    // rest: Sum_k f*_k = p_h (the equilibrium keeps p_h, the forcing sums to 0)
                    if constexpr (FEEDBACK) push(IC<0>{}, IC<0>{}, FLT{}, p_h - stored_sum(IC<0>{}, FLT{}, dev));
                    else push(IC<0>{}, IC<0>{}, FLT{}, keep * fpop[0] + C(FL::w(0)) * (A - g0 * uFh));
                    } else {
                        // TRT: the viscosity sets the symmetric rate w+ = wf; w- from the
                        // magic parameter, 1/w- - 1/2 = Lambda_f / (1/wf - 1/2) = Lambda_f / (3 nu)
                        const C wm = rcp<C>(C(0.5) + KC(P.trt_lf, P.f32.trt_lf) * rcp<C>(C(3) * nu));
                        // shifted equilibrium (feq - F_k/2) and source F_k of direction k
                        auto eqsrc = [&](auto kc, C& eqs, C& Fk) __attribute__((always_inline)) {
                            constexpr int k = decltype(kc)::value;
                            constexpr int ex = FL::ex(k), ey = FL::ey(k), ez = FL::ez(k);
                            const C wk = C(FL::w(k));
                            const C eu = edot<ex, ey, ez>(u[0], u[1], u[2]);
                            const C eF = edot<ex, ey, ez>(F[0], F[1], F[2]);
                            Fk = wk * (g0 + eu * (C(3) + C(4.5) * eu)) * (eF - uF);
                            if constexpr (VD) Fk *= fsc;
                            eqs = wk * (e0 + rho0 * eu * (C(1) + C(1.5) * eu)) - C(0.5) * Fk;
                        };
                        C res = C(0), rest = C(0);
                        static_for<0, QF>([&](auto kc) __attribute__((always_inline)) {
                            constexpr int k = decltype(kc)::value;
                            constexpr int o = FL::opp(k);
                            if constexpr (k == 0) {
                                C eqs, Fk;
                                eqsrc(kc, eqs, Fk);
                                rest = fpop[0] - wf * (fpop[0] - eqs) + Fk;
                                if constexpr (!FEEDBACK) push(kc, kc, FLT{}, rest);
                            } else if constexpr (k < o) {
                                C eqk, Fk, eqo, Fo;
                                eqsrc(kc, eqk, Fk);
                                eqsrc(IC<o>{}, eqo, Fo);
                                const C nk = fpop[k] - eqk, no = fpop[o] - eqo;
                                const C sp = wf * C(0.5) * (nk + no), sm = wm * C(0.5) * (nk - no);
                                push_r(kc, kc, FLT{}, fpop[k] - sp - sm + Fk, res);
                                push_r(IC<o>{}, IC<o>{}, FLT{}, fpop[o] - sp + sm + Fo, res);
                            }
                        });
                        if constexpr (FEEDBACK) push(IC<0>{}, IC<0>{}, FLT{}, rest + fb(IC<0>{}, res));
                    }
                }

                LBM_FENCE();
                // ---- g: Eqs. LBE_Phi, Geq, Source_LBE_Phi ----
                // g* = (1 - w) g + w w_k phi (1 + eu / c_s^2) + (1 - w/2) w_k S
                {
                    const C wg = KC(P.omega_g, P.f32.omega_g);
                    const C keep = C(1) - wg;
                    const C wphi = wg * phi;
                    const C srcS = (C(1) - C(0.5) * wg) * C(m.S);
                    if constexpr (MRTC) {
                        // MRT: the first order (diffusive flux) at the M_phi rate, orders 0
                        // and 2 at the given even rate, third and fourth at theirs
                        const C S = C(m.S), hS = C(0.5) * C(m.S);
                        C resm = C(0), restm = C(0);
                        mrt_relax<SL>(g,
                            [&](auto kc) __attribute__((always_inline)) -> C {
                                constexpr int k = decltype(kc)::value;
                                constexpr int ex = SL::ex(k), ey = SL::ey(k), ez = SL::ez(k);
                                const C wk = C(SL::w(k));
                                if constexpr (ex != 0 || ey != 0 || ez != 0)
                                    return wk * (phi * (C(1) + edot<ex, ey, ez>(u[0], u[1], u[2]) * inv_cs2s) - hS);
                                else
                                    return wk * (phi - hS);
                            },
                            [&](auto kc) __attribute__((always_inline)) -> C { return C(SL::w(decltype(kc)::value)) * S; },
                            [&](auto ic) __attribute__((always_inline)) -> C {
                                constexpr int o = basis_order<SL, decltype(ic)::value>();
                                if constexpr (o == 1) return wg;
                                else if constexpr (o == 3) return KC(P.mrt_s[1], P.f32.mrt_s[1]);
                                else if constexpr (o == 4) return KC(P.mrt_s[2], P.f32.mrt_s[2]);
                                else return KC(P.mrt_s[0], P.f32.mrt_s[0]);
                            },
                            [&](auto kc, C v) __attribute__((always_inline)) {
                                if constexpr (decltype(kc)::value == 0 && FEEDBACK) restm = v;
                                else push_r(IC<G0 + decltype(kc)::value>{}, kc, SLT{}, v, resm);
                            });
                        if constexpr (FEEDBACK) push(IC<G0>{}, IC<0>{}, SLT{}, restm + fb(IC<1>{}, resm));
                    } else if constexpr (!TRTC) {
                    // g*_k = keep g_k + w_k (t + c eu), t = w phi + (1 - w/2) S, c = w phi / c_s^2
                    const C t = wphi + srcS, cu = wphi * inv_cs2s;
                    C dev = C(0);
                    static_for<1, QS>([&](auto kc) __attribute__((always_inline)) {
                        constexpr int k = decltype(kc)::value;
                        constexpr int o = SL::opp(k);
                        if constexpr (k < o) {
                            constexpr int ex = SL::ex(k), ey = SL::ey(k), ez = SL::ez(k);
                            const C wk = C(SL::w(k));
                            const C ceu = cu * edot<ex, ey, ez>(u[0], u[1], u[2]);
                            push_d2(IC<G0 + k>{}, IC<G0 + o>{}, kc, IC<o>{}, SLT{}, keep * g[k] + wk * (t + ceu),
                                    keep * g[o] + wk * (t - ceu), dev);
                        }
                    });
                    // rest: Sum_k g*_k = (1 - w) phi* + w phi + (1 - w/2) S with phi* = Sum_k g_k
                    // (phi = phi* + S*/2 takes the predictor's S*, the source the corrected S)
                    if constexpr (FEEDBACK) {
                        const double wgd = double(wg);
                        const double mg = c_ps + wgd * (m.phi - c_ps) + (1.0 - 0.5 * wgd) * m.S;
                        push(IC<G0>{}, IC<0>{}, SLT{}, C(mg) - stored_sum(IC<1>{}, SLT{}, dev));
                    }
                    else
                        push(IC<G0>{}, IC<0>{}, SLT{}, keep * g[0] + C(SL::w(0)) * t);
                    } else {
                        // TRT: M_phi sets the antisymmetric rate w- = wg; w+ (uniform) from
                        // the magic parameter on the host.  Shifted equilibrium
                        // w_k phi (1 + eu / c_s^2) - w_k S / 2, source w_k S.
                        const C wp = KC(P.omega_gp, P.f32.omega_gp);
                        const C S = C(m.S), hS = C(0.5) * C(m.S);
                        auto eqs = [&](auto kc) __attribute__((always_inline)) -> C {
                            constexpr int k = decltype(kc)::value;
                            constexpr int ex = SL::ex(k), ey = SL::ey(k), ez = SL::ez(k);
                            const C wk = C(SL::w(k));
                            if constexpr (ex != 0 || ey != 0 || ez != 0)
                                return wk * (phi * (C(1) + edot<ex, ey, ez>(u[0], u[1], u[2]) * inv_cs2s) - hS);
                            else
                                return wk * (phi - hS);
                        };
                        C res = C(0), rest = C(0);
                        static_for<0, QS>([&](auto kc) __attribute__((always_inline)) {
                            constexpr int k = decltype(kc)::value;
                            constexpr int o = SL::opp(k);
                            if constexpr (k == 0) {
                                rest = g[0] - wp * (g[0] - eqs(kc)) + C(SL::w(0)) * S;
                                if constexpr (!FEEDBACK) push(IC<G0>{}, kc, SLT{}, rest);
                            } else if constexpr (k < o) {
                                const C nk = g[k] - eqs(kc), no = g[o] - eqs(IC<o>{});
                                const C sp = wp * C(0.5) * (nk + no), sm = wg * C(0.5) * (nk - no);
                                push_r(IC<G0 + k>{}, kc, SLT{}, g[k] - sp - sm + C(SL::w(k)) * S, res);
                                push_r(IC<G0 + o>{}, IC<o>{}, SLT{}, g[o] - sp + sm + C(SL::w(o)) * S, res);
                            }
                        });
                        if constexpr (FEEDBACK) push(IC<G0>{}, IC<0>{}, SLT{}, rest + fb(IC<1>{}, res));
                    }
                }

                LBM_FENCE();
                // ---- h^A, h^B: Eqs. LBE_c_alpha, Heq; mobility interpolated in phi ----
                {
                    const C MA = KC(P.MA0, P.f32.MA0) * (C(1) - phi) + KC(P.MA1, P.f32.MA1) * phi;
                    const C MB = KC(P.MB0, P.f32.MB0) * (C(1) - phi) + KC(P.MB1, P.f32.MB1) * phi;
                    const C wA = rcp<C>(MA * inv_cs2s + C(0.5));
                    const C wB = rcp<C>(MB * inv_cs2s + C(0.5));
                    if constexpr (MRTC) {
                        // MRT: the first order at the mobility rate, the others at the given
                        // rates (order 0 with the even rate: c is conserved exactly)
                        auto rates = [&](C wflux) __attribute__((always_inline)) {
                            return [&, wflux](auto ic) __attribute__((always_inline)) -> C {
                                constexpr int o = basis_order<SL, decltype(ic)::value>();
                                if constexpr (o == 1) return wflux;
                                else if constexpr (o == 3) return KC(P.mrt_s[1], P.f32.mrt_s[1]);
                                else if constexpr (o == 4) return KC(P.mrt_s[2], P.f32.mrt_s[2]);
                                else return KC(P.mrt_s[0], P.f32.mrt_s[0]);
                            };
                        };
                        auto heq = [&](double c, double mu) __attribute__((always_inline)) {
                            return [&, c, mu](auto kc) __attribute__((always_inline)) -> C {
                                constexpr int k = decltype(kc)::value;
                                constexpr int ex = SL::ex(k), ey = SL::ey(k), ez = SL::ez(k);
                                if constexpr (k == 0) return C(c - (1.0 - SL::w(0)) * mu);
                                else return C(SL::w(k)) * (C(mu) + C(c) * edot<ex, ey, ez>(u[0], u[1], u[2]) * inv_cs2s);
                            };
                        };
                        auto zero = [&](auto) __attribute__((always_inline)) -> C { return C(0); };
                        C resA = C(0), restA = C(0), resB = C(0), restB = C(0);
                        mrt_relax<SL>(a, heq(sA, m.muA), zero, rates(wA),
                                      [&](auto kc, C v) __attribute__((always_inline)) {
                                          if constexpr (decltype(kc)::value == 0 && FEEDBACK) restA = v;
                                          else push_r(IC<A0 + decltype(kc)::value>{}, kc, SLT{}, v, resA);
                                      });
                        mrt_relax<SL>(b, heq(sB, m.muB), zero, rates(wB),
                                      [&](auto kc, C v) __attribute__((always_inline)) {
                                          if constexpr (decltype(kc)::value == 0 && FEEDBACK) restB = v;
                                          else push_r(IC<B0 + decltype(kc)::value>{}, kc, SLT{}, v, resB);
                                      });
                        if constexpr (FEEDBACK) {
                            push(IC<A0>{}, IC<0>{}, SLT{}, restA + fb(IC<2>{}, resA));
                            push(IC<B0>{}, IC<0>{}, SLT{}, restB + fb(IC<3>{}, resB));
                        }
                    } else if constexpr (TRTC) {
                        // TRT: the mobility sets the antisymmetric rate w- = wA (wB); w+ from
                        // the magic parameter, 1/w+ - 1/2 = Lambda_s / (M / c_s^2)
                        const C ls = KC(P.trt_ls, P.f32.trt_ls);
                        const C wpA = rcp<C>(C(0.5) + ls * rcp<C>(MA * inv_cs2s));
                        const C wpB = rcp<C>(C(0.5) + ls * rcp<C>(MB * inv_cs2s));
                        // rest populations (symmetric) in double, as in BGK, stored last with
                        // the rounding residues of 16-bit storage
                        const double pa = double(a[0]) - double(wpA) * (double(a[0]) - (sA - (1.0 - SL::w(0)) * m.muA));
                        const double pb = double(b[0]) - double(wpB) * (double(b[0]) - (sB - (1.0 - SL::w(0)) * m.muB));
                        C resA = C(0), resB = C(0);
                        const C muA = C(m.muA), muB = C(m.muB);
                        const C cuA = C(sA) * inv_cs2s, cuB = C(sB) * inv_cs2s;
                        static_for<1, QS>([&](auto kc) __attribute__((always_inline)) {
                            constexpr int k = decltype(kc)::value;
                            constexpr int o = SL::opp(k);
                            if constexpr (k < o) {
                                constexpr int ex = SL::ex(k), ey = SL::ey(k), ez = SL::ez(k);
                                const C wk = C(SL::w(k));  // w_opp(k) = w_k
                                const C eu = edot<ex, ey, ez>(u[0], u[1], u[2]);  // e_opp . u = -eu
                                // h^eq_k = w_k (mu + c eu / c_s^2): symmetric part w_k mu, antisymmetric w_k c eu / c_s^2
                                const C npA = C(0.5) * (a[k] + a[o]) - wk * muA, nmA = C(0.5) * (a[k] - a[o]) - wk * cuA * eu;
                                const C npB = C(0.5) * (b[k] + b[o]) - wk * muB, nmB = C(0.5) * (b[k] - b[o]) - wk * cuB * eu;
                                push_r(IC<A0 + k>{}, kc, SLT{}, a[k] - wpA * npA - wA * nmA, resA);
                                push_r(IC<A0 + o>{}, IC<o>{}, SLT{}, a[o] - wpA * npA + wA * nmA, resA);
                                push_r(IC<B0 + k>{}, kc, SLT{}, b[k] - wpB * npB - wB * nmB, resB);
                                push_r(IC<B0 + o>{}, IC<o>{}, SLT{}, b[o] - wpB * npB + wB * nmB, resB);
                            }
                        });
                        push(IC<A0>{}, IC<0>{}, SLT{}, C(pa + double(fb(IC<2>{}, resA))));
                        push(IC<B0>{}, IC<0>{}, SLT{}, C(pb + double(fb(IC<3>{}, resB))));
                    } else {
                    // BGK: h*_k = keep h_k + w_k (w mu + w c eu / c_s^2); k and opp(k) share w mu.
                    // Rest populations in double (they carry the conserved composition): from
                    // the collision with FP32 / FP64 storage, as c minus the stored moving
                    // populations with 16-bit storage
                    const C keepA = C(1) - wA, keepB = C(1) - wB;
                    const C wmuA = wA * C(m.muA), wmuB = wB * C(m.muB);
                    const C wcA = wA * C(sA) * inv_cs2s, wcB = wB * C(sB) * inv_cs2s;
                    C devA = C(0), devB = C(0);
                    // a third composition: the same BGK relaxation with its own mobility
                    C wC = C(0), keepC = C(0), wmuC = C(0), wcC = C(0), devC = C(0);
                    if constexpr (NC3) {
                        const C MC = KC(P.MC0, P.f32.MC0) * (C(1) - phi) + KC(P.MC1, P.f32.MC1) * phi;
                        wC = rcp<C>(MC * inv_cs2s + C(0.5));
                        keepC = C(1) - wC;
                        wmuC = wC * C(muC);
                        wcC = wC * C(sC) * inv_cs2s;
                    }
                    static_for<1, QS>([&](auto kc) __attribute__((always_inline)) {
                        constexpr int k = decltype(kc)::value;
                        constexpr int o = SL::opp(k);
                        if constexpr (k < o) {
                            constexpr int ex = SL::ex(k), ey = SL::ey(k), ez = SL::ez(k);
                            const C wk = C(SL::w(k));  // w_opp(k) = w_k
                            const C eu = edot<ex, ey, ez>(u[0], u[1], u[2]);
                            push_d2(IC<A0 + k>{}, IC<A0 + o>{}, kc, IC<o>{}, SLT{}, keepA * a[k] + wk * (wmuA + wcA * eu),
                                    keepA * a[o] + wk * (wmuA - wcA * eu), devA);
                            push_d2(IC<B0 + k>{}, IC<B0 + o>{}, kc, IC<o>{}, SLT{}, keepB * b[k] + wk * (wmuB + wcB * eu),
                                    keepB * b[o] + wk * (wmuB - wcB * eu), devB);
                            if constexpr (NC3)
                                push_d2(IC<HC0 + k>{}, IC<HC0 + o>{}, kc, IC<o>{}, SLT{},
                                        keepC * cq[k] + wk * (wmuC + wcC * eu), keepC * cq[o] + wk * (wmuC - wcC * eu),
                                        devC);
                        }
                    });
                    if constexpr (FEEDBACK) {
                        push(IC<A0>{}, IC<0>{}, SLT{}, C(sA - double(stored_sum(IC<2>{}, SLT{}, devA))));
                        push(IC<B0>{}, IC<0>{}, SLT{}, C(sB - double(stored_sum(IC<3>{}, SLT{}, devB))));
                        if constexpr (NC3)
                            push(IC<HC0>{}, IC<0>{}, SLT{}, C(sC - double(stored_sum(IC<4>{}, SLT{}, devC))));
                    } else {
                        const double w1 = 1.0 - SL::w(0);
                        auto rest = [&](C h0, C w, double sc, double mu) __attribute__((always_inline)) -> C {
                            return C(double(h0) - double(w) * (double(h0) - (sc - w1 * mu)));
                        };
                        push(IC<A0>{}, IC<0>{}, SLT{}, rest(a[0], wA, sA, m.muA));
                        push(IC<B0>{}, IC<0>{}, SLT{}, rest(b[0], wB, sB, m.muB));
                        if constexpr (NC3) push(IC<HC0>{}, IC<0>{}, SLT{}, rest(cq[0], wC, sC, muC));
                    }
                    }
                }

            } else if constexpr (MODE == MODE_MOMENTS) {
                // hydrodynamic pressure: p_h, or rho c_s^2 p* with variable density
                const double p_out = VD ? double(p_h) / (3.0 * double(irho)) : double(p_h);
                const double vals[kNumMom] = {m.phi, sA, sB, m.muA, m.muB, p_out,
                                              double(u[0]), double(u[1]), double(u[2]), sC, muC};
                constexpr int NMOM = NC3 ? kNumMom : kNumMom - 2;
#pragma unroll
                for (int i = 0; i < NMOM; ++i) {
                    if (P.mout[i]) {
                        if (P.mout_f32) static_cast<float*>(P.mout[i])[idx] = float(vals[i]);
                        else static_cast<double*>(P.mout[i])[idx] = vals[i];
                    }
                }
            } else {  // MODE_DIAG
                const double u2 = double(u[0]) * double(u[0]) + double(u[1]) * double(u[1]) +
                                  double(u[2]) * double(u[2]);
                const double g2 = double(grad[0]) * double(grad[0]) + double(grad[1]) * double(grad[1]) +
                                  double(grad[2]) * double(grad[2]);
                acc[0] += sA;
                acc[1] += sB;
                acc[2] += m.phi;
                acc[3] += 0.5 * (VD ? P.rho0 + P.drho * m.phi : P.rho0) * u2;
                acc[4] = fmax(acc[4], sqrt(u2));
                acc[5] += (4.0 / P.W) * m.phi * (1.0 - m.phi);
                if constexpr (NC3) {
                    acc[6] += 0.5 * P.W * P.W * g2 + dwell(m.phi) +
                              P.lam * 0.5 * (m.muA * m.muA + m.muB * m.muB + muC * muC);
                    acc[7] += (isfinite(m.phi) && isfinite(sA) && isfinite(sB) && isfinite(sC)) ? 0.0 : 1.0;
                    acc[NACC - 1] += sC;
                } else {
                    acc[6] += 0.5 * P.W * P.W * g2 + dwell(m.phi) + P.lam * bulk_free_energy<GK>(m.phi, m.muA, m.muB, P);
                    acc[7] += (isfinite(m.phi) && isfinite(sA) && isfinite(sB)) ? 0.0 : 1.0;
                }
                P.mask_out[idx] = m.phi >= 0.5 ? 1 : 0;
            }
        }
        if constexpr (STENCIL) {
            // the next plane becomes the current one
            if constexpr (!LDS_POPS) {
#pragma unroll
                for (int k = 0; k < QS; ++k) { cg[k] = ng[k]; ca[k] = na[k]; cb[k] = nb[k]; }
                if constexpr (NC3) {
#pragma unroll
                    for (int k = 0; k < QS; ++k) cq[k] = nq[k];
                }
            }
            c_ps = n_ps; c_cA = n_cA; c_cB = n_cB; c_cC = n_cC;
            __syncthreads();
        }
    }

    if constexpr (MODE == MODE_DIAG) {
        block_reduce_store<NACC, NT>(acc, 4, P.partials + NACC * tile);
    } else if constexpr (MODE == MODE_STEP || MODE == MODE_STEP_PHI) {
        if (P.mean_subtract) block_reduce_store<1, NT>(acc, -1, P.partials + tile);
    }
}

// ---------------------------------------------------------------------------
// half-way bounce-back as a fix-up between steps (Section 4.2.4: walls at rest
// with zero normal flux).  The next step pulls X_k(x) from slot k at
// wrap(x - e_k).  When x - e_k lies across a wall, bounce-back wants instead the
// post-collision population that left x towards the wall, slot opp(k) at x.
// Node x' = wrap(x - e_k) is in the mirror situation: it pulls slot opp(k) at x
// and wants its own slot k.  Exchanging the two entries serves both.  Each
// exchange is done once, by the node x and direction k with k < opp(k); each
// wall node is visited by exactly one thread: the face of its lowest-index wall
// axis.

template <class SL, class FL, int PREC, int NC = 2>
__global__ void __launch_bounds__(256) k_walls(const KParams P, int axis) {
    using SLOTS = Slots<FL::Q, SL::Q, NC>;
    // enumerate the two faces of `axis`: (b, c) span the other two axes
    const int n[3] = {P.nx, P.ny, P.nz};
    const int ab = axis == 0 ? 1 : 0, ac = axis == 2 ? 1 : 2;
    const long long face = (long long)n[ab] * n[ac];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * face) return;
    int c[3];
    c[axis] = t < face ? 0 : n[axis] - 1;
    const long long r = t % face;
    c[ab] = int(r % n[ab]);
    c[ac] = int(r / n[ab]);
    // walls on x and y only: the z walls bounce back when the next step pulls
    const int wall[3] = {P.wall_x, P.wall_y, 0};
    // skip nodes owned by the face of a lower wall axis
    for (int a = 0; a < axis; ++a)
        if (wall[a] && (c[a] == 0 || c[a] == n[a] - 1)) return;
    if (n[axis] == 1 && t >= face) return;  // both faces are the same plane
    const int idx = (c[2] * P.ny + c[1]) * P.nx + c[0];

    // does x - e lie across an x or y wall (and not across a z wall, which the pull
    // handles)?
    auto crosses = [&](int ex, int ey, int ez) {
        if (P.wall_z && ez != 0 && (c[2] - ez < 0 || c[2] - ez >= n[2])) return false;
        const int e[3] = {ex, ey, ez};
        for (int a = 0; a < 3; ++a)
            if (wall[a] && e[a] != 0 && (c[a] - e[a] < 0 || c[a] - e[a] >= n[a])) return true;
        return false;
    };
    // index of wrap(x - e)
    auto source = [&](int ex, int ey, int ez) {
        const int e[3] = {ex, ey, ez};
        int q[3];
        for (int a = 0; a < 3; ++a) q[a] = (c[a] - e[a] + n[a]) % n[a];
        return (q[2] * P.ny + q[1]) * P.nx + q[0];
    };
    // raw storage word of slot S at node i
    using Word = typename std::conditional<PREC == P64, double,
                                           typename std::conditional<PREC == P32, float, unsigned short>::type>::type;
    auto word = [&](auto s_, int i) -> Word* {
        constexpr int S = decltype(s_)::value;
        return reinterpret_cast<Word*>(P.dst_base + slot_offset<SLOTS, S>(P)) + i;
    };
    // every exchange pair (slot k at wrap(x - e_k), slot opp(k) at x), k < opp(k);
    // 16-bit formats: moving populations only (equal references for k and opp(k))
    auto pairs = [&](auto&& fn) {
        auto lattice = [&](auto lat_, auto base_) {
            using L = typename decltype(lat_)::type;
            constexpr int B = decltype(base_)::value;
            static_for<1, L::Q>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                constexpr int o = L::opp(k);
                if constexpr (k < o) fn(IC<B + k>{}, IC<B + o>{}, IC<L::ex(k)>{}, IC<L::ey(k)>{}, IC<L::ez(k)>{});
            });
        };
        if constexpr (FL::Q > 0) lattice(std::common_type<FL>{}, IC<0>{});
        lattice(std::common_type<SL>{}, IC<SLOTS::G0>{});
        lattice(std::common_type<SL>{}, IC<SLOTS::A0>{});
        lattice(std::common_type<SL>{}, IC<SLOTS::B0>{});
        if constexpr (NC >= 3) lattice(std::common_type<SL>{}, IC<SLOTS::C0>{});
    };
    constexpr int NP = (FL::Q > 0 ? (FL::Q - 1) / 2 : 0) + (1 + NC) * ((SL::Q - 1) / 2);
    // all loads first, then all stores: the round trips overlap
    Word va[NP], vb[NP];
    bool cr[NP];
    int np = 0;
    pairs([&](auto s_, auto o_, auto ex_, auto ey_, auto ez_) {
        const int p = np++;
        cr[p] = crosses(ex_.value, ey_.value, ez_.value);
        if (cr[p]) {
            va[p] = *word(s_, source(ex_.value, ey_.value, ez_.value));
            vb[p] = *word(o_, idx);
        }
    });
    np = 0;
    pairs([&](auto s_, auto o_, auto ex_, auto ey_, auto ez_) {
        const int p = np++;
        if (cr[p]) {
            *word(s_, source(ex_.value, ey_.value, ez_.value)) = vb[p];
            *word(o_, idx) = va[p];
        }
    });
}

// ---------------------------------------------------------------------------
// initialisation at rest (Section 4.2.1): equilibrium populations from (phi_0, mu_0).
// A copy holds post-collision populations at the node that computed them; the
// next step pulls X_k(x) from slot k at wrap(x - e_k).  The equilibrium X_k(x) is
// therefore written to slot k at wrap(x - e_k).

template <class SL, class FL, int PREC, int NC = 2>
__global__ void __launch_bounds__(256) k_init(const KParams P, const double* __restrict__ phi0,
                                              const double* __restrict__ muA0,
                                              const double* __restrict__ muB0,
                                              const double* __restrict__ muC0) {
    using C = typename Stor<PREC>::C;
    using SLOTS = Slots<FL::Q, SL::Q, NC>;
    constexpr int G0 = SLOTS::G0, A0 = SLOTS::A0, B0 = SLOTS::B0, HC0 = SLOTS::C0;
    using STL = typename std::conditional<SL::DIM == 2, D2Q9K, D3Q19K>::type;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= P.nx) return;
    const int idx = (z * P.ny + y) * P.nx + x;
    const Nbr nb = neighbours(x, y, z, P);
    const double phi = phi0[idx], muA = muA0[idx], muB = muB0[idx];
    const double pp = interp_p(phi);
    // Eq. species_closure (general curvatures: c = c^eq(phi) + kappa(phi) mu), unless the
    // compositions are given (initial condition of Section 4.2.1: c stepped at phi = 1/2
    // with mu = 0)
    double kA = muA, kB = muB;  // kappa(phi) mu
    double domega = -(muA * (P.c0A - P.c1A) + muB * (P.c0B - P.c1B));
    if (P.general_k) {
        const double kAA = P.kap0[0] + pp * (P.kap1[0] - P.kap0[0]);
        const double kAB = P.kap0[1] + pp * (P.kap1[1] - P.kap0[1]);
        const double kBB = P.kap0[2] + pp * (P.kap1[2] - P.kap0[2]);
        kA = kAA * muA + kAB * muB;
        kB = kAB * muA + kBB * muB;
        const double dAA = P.kap0[0] - P.kap1[0], dAB = P.kap0[1] - P.kap1[1], dBB = P.kap0[2] - P.kap1[2];
        domega -= 0.5 * (dAA * muA * muA + 2.0 * dAB * muA * muB + dBB * muB * muB);
    }
    const double cA = P.init_c[0] ? P.init_c[0][idx] : kA + P.c0A + pp * (P.c1A - P.c0A);
    const double cB = P.init_c[1] ? P.init_c[1][idx] : kB + P.c0B + pp * (P.c1B - P.c0B);
    // a third composition: the same closure, and its share of Delta omega
    double muC = 0.0, cC = 0.0;
    if constexpr (NC >= 3) {
        muC = muC0[idx];
        cC = P.init_c[2] ? P.init_c[2][idx] : muC + P.c0C + pp * (P.c1C - P.c0C);
        domega -= muC * (P.c0C - P.c1C);
    }
    const double S0 = P.mphi_w2 * (P.lam * interp_dp(phi) * domega - dwell_d(phi));

    // returns the rounding residue (value - stored value); 16-bit storage adds the
    // residues of a field's moving populations to its rest population, written last
    auto put = [&](auto s_, auto k_, auto lat_, double v) -> double {
        using L = typename decltype(lat_)::type;
        constexpr int S = decltype(s_)::value, k = decltype(k_)::value;
        constexpr int F = SLOTS::field(S);
        unsigned t;
        char* slot = const_cast<char*>(pull_src<SLOTS, L, S, k>(P.dst_base, P, z, unsigned(idx), nb, t));
        return v - double(st_at_r<PREC, SLOTS::rest(S)>(slot, t, float(L::w(k)) * P.fref[F], P.fscale[F],
                                                         P.finv[F], C(v)));
    };
    double rg = 0.0, ra = 0.0, rb = 0.0, rc = 0.0;
    static_for<1, SL::Q>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr double wk = SL::w(k);
        rg += put(IC<G0 + k>{}, kc, std::common_type<SL>{}, wk * phi - 0.5 * wk * S0);
        ra += put(IC<A0 + k>{}, kc, std::common_type<SL>{}, wk * muA);
        rb += put(IC<B0 + k>{}, kc, std::common_type<SL>{}, wk * muB);
        if constexpr (NC >= 3) rc += put(IC<HC0 + k>{}, kc, std::common_type<SL>{}, wk * muC);
    });
    {
        constexpr double w0 = SL::w(0);
        put(IC<G0>{}, IC<0>{}, std::common_type<SL>{}, w0 * phi - 0.5 * w0 * S0 + rg);
        put(IC<A0>{}, IC<0>{}, std::common_type<SL>{}, cA - (1.0 - w0) * muA + ra);
        put(IC<B0>{}, IC<0>{}, std::common_type<SL>{}, cB - (1.0 - w0) * muB + rb);
        if constexpr (NC >= 3) put(IC<HC0>{}, IC<0>{}, std::common_type<SL>{}, cC - (1.0 - w0) * muC + rc);
    }
    if constexpr (FL::Q > 0) {
        double grad[3] = {0.0, 0.0, 0.0}, lap = 0.0;
#pragma unroll
        for (int k = 1; k < STL::Q; ++k) {
            const int xn = map_coord(x + STL::ex(k), P.nx, P.wall_x);
            const int yn = map_coord(y + STL::ey(k), P.ny, P.wall_y);
            const int zn = map_coord(z + STL::ez(k), P.nz, P.wall_z);
            const double v = phi0[(zn * P.ny + yn) * P.nx + xn];
            grad[0] += 3.0 * STL::w(k) * STL::ex(k) * v;
            grad[1] += 3.0 * STL::w(k) * STL::ey(k) * v;
            grad[2] += 3.0 * STL::w(k) * STL::ez(k) * v;
            lap += 6.0 * STL::w(k) * (v - phi);
        }
        const double phi_ref = P.mean_subtract ? *P.phi_ref : 0.0;
        const double bracket = P.cap * (dwell_d(phi) * P.inv_W2 - lap);
        const double buoy = (phi - phi_ref) * P.drho;
        const double F[3] = {buoy * P.gx + bracket * grad[0], buoy * P.gy + bracket * grad[1],
                             buoy * P.gz + bracket * grad[2]};
        double rf = 0.0;
        // variable density: dimensionless populations, forcing divided by rho(phi) c_s^2
        const double fsc = P.variable_density ? 3.0 / (P.rho0 + P.drho * phi) : 1.0;
        static_for<1, FL::Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const double eF = (FL::ex(k) * F[0] + FL::ey(k) * F[1] + FL::ez(k) * F[2]) * fsc;
            // f^eq at p_h = 0, u = 0 minus F_k / 2 with Gamma_k(u = 0) = w_k
            rf += put(kc, kc, std::common_type<FL>{}, -0.5 * FL::w(k) * eF);
        });
        put(IC<0>{}, IC<0>{}, std::common_type<FL>{}, rf);  // e_0 . F = 0
    }
}

// ---------------------------------------------------------------------------
// canonical FP64 population access: X_k(x) lives in slot k at wrap(x - e_k)

template <class SL, class FL, int PREC, bool SET, int NC = 2>
__global__ void __launch_bounds__(256) k_pops(const KParams P, long long nodes, double* __restrict__ buf) {
    using C = typename Stor<PREC>::C;
    using SLOTS = Slots<FL::Q, SL::Q, NC>;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nodes) return;
    const int x = int(i % P.nx), y = int((i / P.nx) % P.ny), z = int(i / ((long long)P.nx * P.ny));
    const Nbr nb = neighbours(x, y, z, P);
    auto one = [&](auto s_, auto k_, auto lat_) {
        using L = typename decltype(lat_)::type;
        constexpr int S = decltype(s_)::value, k = decltype(k_)::value;
        const float wref = float(L::w(k)) * P.fref[SLOTS::field(S)];
        unsigned t;
        if constexpr (SET) {
            char* slot = const_cast<char*>(pull_src<SLOTS, L, S, k>(P.dst_base, P, z, unsigned(i), nb, t));
            st_at<PREC, SLOTS::rest(S)>(slot, t, wref, P.fscale[SLOTS::field(S)], C(buf[S * nodes + i]));
        } else {
            const char* slot = pull_src<SLOTS, L, S, k>(P.src_base, P, z, unsigned(i), nb, t);
            buf[S * nodes + i] = double(ld_at<PREC, SLOTS::rest(S)>(slot, t, wref, P.finv[SLOTS::field(S)]));
        }
    };
    static_for<0, FL::Q>([&](auto kc) { one(kc, kc, std::common_type<FL>{}); });
    static_for<0, SL::Q>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        one(IC<SLOTS::G0 + k>{}, kc, std::common_type<SL>{});
        one(IC<SLOTS::A0 + k>{}, kc, std::common_type<SL>{});
        one(IC<SLOTS::B0 + k>{}, kc, std::common_type<SL>{});
        if constexpr (NC >= 3) one(IC<SLOTS::C0 + k>{}, kc, std::common_type<SL>{});
    });
}

// ---------------------------------------------------------------------------
// adjoint kernels.  The adjoint of the arriving population X_s(x) is lambda_s(x)
// (FP32 [slot][node], P.adj_in / P.adj_out) plus c_F(x) (rows of P.auxc) when s is a
// scalar population of field F.  Kernels over nodes use 256-thread work-groups; their
// theta partials accumulate in P.partials + 6 * blockIdx.x.

template <class SL, class FL>
__device__ __forceinline__ float* adj_at(const char* base, const KParams& P, int slot, unsigned long long idx) {
    return reinterpret_cast<float*>(const_cast<char*>(base) + (unsigned long long)slot * P.adj_stride + idx * 4u);
}

__device__ __forceinline__ void theta_from_K(double K_b, const KParams& P, double (&th)[6]) {
    // K = M_phi / W^2
    th[0] += K_b / (P.W * P.W);
    th[5] += K_b * (-2.0 * P.mphi_w2 / P.W);
}

// Adjoint of one step, one thread per node.  mu = dL/dQ(x) is the transposed
// streaming of the adjoint of step n + 1: mu_k(x) = Lambda_k(x + e_k), or
// Lambda_opp(k)(x) when x + e_k lies across a wall (bounce-back), where Lambda =
// lambda (+ c_F for scalar fields).  The arriving populations of state n are pulled
// as in the step; the phi stencil reads phi of state n (`phi`, written by the step
// that left state n).  lambda^n gets the local part (P.adj_out); dL/dG, dL/dN and the
// sensitivities of phi go to aux rows 0..6 for k_adj_gather; theta partials
// accumulate per work-group.
template <class SL, class FL, int PREC>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(SL::DIM == 2 ? LBM_ADJ_WAVES_2D : LBM_ADJ_WAVES_3D)))
k_adj_node(const KParams P, long long nodes, const typename Stor<PREC>::C* __restrict__ phi) {
    using C = typename Stor<PREC>::C;
    using T = C;
    using SLOTS = Slots<FL::Q, SL::Q>;
    using STL = typename std::conditional<SL::DIM == 2, D2Q9K, D3Q19K>::type;
    constexpr int QS = SL::Q, QF = FL::Q;
    constexpr int G0 = SLOTS::G0, A0 = SLOTS::A0, B0 = SLOTS::B0;
    using SLT = std::common_type<SL>;
    using FLT = std::common_type<FL>;
    // 32-bit node index (nodes < 2^31): keeps every access in the voffset + saddr form
    const unsigned idx = blockIdx.x * 256u + threadIdx.x;
    double th[6] = {0, 0, 0, 0, 0, 0};
    if (idx < (unsigned long long)nodes) {
        const unsigned nxny = unsigned(P.nx) * unsigned(P.ny);
        const int z = int(idx / nxny), r = int(idx - unsigned(z) * nxny);
        const int y = r / P.nx, x = r - y * P.nx;
        const Nbr nbr = neighbours(x, y, z, P);
        auto load = [&](auto s_, auto k_, auto lat_) __attribute__((always_inline)) -> C {
            using L = typename decltype(lat_)::type;
            constexpr int S = decltype(s_)::value, k = decltype(k_)::value;
            unsigned t;
            const char* slot = pull_src<SLOTS, L, S, k>(P.src_base, P, z, idx, nbr, t);
            return ld_at<PREC, SLOTS::rest(S)>(slot, t, float(L::w(k)) * P.fref[SLOTS::field(S)],
                                               P.finv[SLOTS::field(S)]);
        };
        C fpop[QF > 0 ? QF : 1], g[QS], a[QS], b[QS];
        static_for<0, QF>([&](auto kc) __attribute__((always_inline)) { fpop[kc.value] = load(kc, kc, FLT{}); });
        static_for<0, QS>([&](auto kc) __attribute__((always_inline)) {
            g[kc.value] = load(IC<G0 + kc.value>{}, kc, SLT{});
            a[kc.value] = load(IC<A0 + kc.value>{}, kc, SLT{});
            b[kc.value] = load(IC<B0 + kc.value>{}, kc, SLT{});
        });
        // phi stencil inputs of Eqs. Grad and Laplacian (mirror ghosts at walls)
        double G[3] = {0.0, 0.0, 0.0}, Nsum = 0.0, pc = 0.0;
        if constexpr (QF > 0) {
            const Nbr sn = stencil_neighbours(x, y, z, P);
            const char* pb = reinterpret_cast<const char*>(phi);
            pc = double(*reinterpret_cast<const C*>(pb + voff(idx * unsigned(sizeof(C)))));
            static_for<1, STL::Q>([&](auto kc) __attribute__((always_inline)) {
                constexpr int k = decltype(kc)::value;
                constexpr int ex = STL::ex(k), ey = STL::ey(k), ez = STL::ez(k);
                const unsigned t = unsigned(int(idx) + push_offset<ex, ey, ez>(sn));
                const double v = double(*reinterpret_cast<const C*>(pb + voff(t * unsigned(sizeof(C))))) *
                                 (3.0 * STL::w(k));
                if constexpr (ex != 0) G[0] += ex > 0 ? v : -v;
                if constexpr (ey != 0) G[1] += ey > 0 ? v : -v;
                if constexpr (ez != 0) G[2] += ez > 0 ? v : -v;
                Nsum += v;
            });
        }
        const float* cin = P.auxc;
        const unsigned own = voff(idx * 4u);
        const bool lo[3] = {P.wall_x && x == 0, P.wall_y && y == 0, P.wall_z && z == 0};
        const bool hi[3] = {P.wall_x && x == P.nx - 1, P.wall_y && y == P.ny - 1, P.wall_z && z == P.nz - 1};
        // mu_s(x) = Lambda_s(wrap(x + e_s)), or Lambda_opp(s)(x) across a wall
        auto mu_of = [&](auto s_) __attribute__((always_inline)) -> T {
            constexpr int S = decltype(s_)::value;
            constexpr bool FLUID = S < G0;
            constexpr int F = FLUID ? -1 : (S - G0) / QS;  // scalar field 0 g, 1 hA, 2 hB
            constexpr int k = FLUID ? S : (S - G0) % QS;
            using L = typename std::conditional<FLUID, FL, SL>::type;
            // wave-uniform bases, 32-bit byte offsets (global_load voffset, saddr)
            const unsigned t = unsigned(int(idx) + push_offset<L::ex(k), L::ey(k), L::ez(k)>(nbr));
            const char* ls = P.adj_in + (unsigned long long)S * P.adj_stride;
            const unsigned o = voff(t * 4u);
            float v = *reinterpret_cast<const float*>(ls + o);
            if constexpr (F >= 0) {
                const char* cf = reinterpret_cast<const char*>(cin + (unsigned long long)F * P.aux_stride);
                v += *reinterpret_cast<const float*>(cf + o);
            }
            return T(v);
        };
        // bounce-back: Lambda_opp(s)(x) at the node itself when x + e_s crosses a wall
        auto mu_wall = [&](auto s_, T& v) __attribute__((always_inline)) {
            constexpr int S = decltype(s_)::value;
            constexpr bool FLUID = S < G0;
            constexpr int F = FLUID ? -1 : (S - G0) / QS;
            constexpr int k = FLUID ? S : (S - G0) % QS;
            using L = typename std::conditional<FLUID, FL, SL>::type;
            constexpr int ex = L::ex(k), ey = L::ey(k), ez = L::ez(k);
            if constexpr (ex != 0 || ey != 0 || ez != 0) {
                bool cross = false;
                if constexpr (ex > 0) cross = cross || hi[0];
                if constexpr (ex < 0) cross = cross || lo[0];
                if constexpr (ey > 0) cross = cross || hi[1];
                if constexpr (ey < 0) cross = cross || lo[1];
                if constexpr (ez > 0) cross = cross || hi[2];
                if constexpr (ez < 0) cross = cross || lo[2];
                if (cross) {
                    constexpr int O = S - k + L::opp(k);
                    const char* lo_ = P.adj_in + (unsigned long long)O * P.adj_stride;
                    float w = *reinterpret_cast<const float*>(lo_ + own);
                    if constexpr (F >= 0)
                        w += *reinterpret_cast<const float*>(
                            reinterpret_cast<const char*>(cin + (unsigned long long)F * P.aux_stride) + own);
                    v = T(w);
                }
            }
        };
        // adjoint of step n + 1 read once into registers: every neighbour load first,
        // then the wall lanes' replacements (a region that other waves skip)
        T muv[SLOTS::N];
        static_for<0, SLOTS::N>([&](auto sc) __attribute__((always_inline)) { muv[sc.value] = mu_of(sc); });
        const bool wall_lane = lo[0] || lo[1] || lo[2] || hi[0] || hi[1] || hi[2];
        if (wall_lane)
            static_for<0, SLOTS::N>([&](auto sc) __attribute__((always_inline)) { mu_wall(sc, muv[sc.value]); });
        auto mu_reg = [&](auto s_) __attribute__((always_inline)) -> T { return muv[decltype(s_)::value]; };
        auto put = [&](auto s_, T v) __attribute__((always_inline)) {
            char* o = P.adj_out + (unsigned long long)decltype(s_)::value * P.adj_stride;
            __builtin_nontemporal_store(float(v), reinterpret_cast<float*>(o + own));
        };
        const double phi_ref = P.mean_subtract ? *P.phi_ref : 0.0;
        double Gb[3], Nb = 0.0;
        node_adjoint<SL, FL, T>(fpop, g, a, b, G, Nsum, pc, phi_ref, P, mu_reg, put, Gb, Nb, th);
        double ps = 0.0, sA = 0.0, sB = 0.0;
        for (int k = 0; k < QS; ++k) { ps += double(g[k]); sA += double(a[k]); sB += double(b[k]); }
        const PhiSens ds = phi_sensitivities(ps, sA, sB, P);
        auto aux_put = [&](int row, double v) __attribute__((always_inline)) {
            char* o = reinterpret_cast<char*>(P.aux + (unsigned long long)row * P.aux_stride);
            *reinterpret_cast<float*>(o + own) = float(v);
        };
        if constexpr (QF > 0) {
            aux_put(0, Gb[0]);
            if constexpr (SL::DIM == 3) aux_put(1, Gb[1]);
            aux_put(2, Gb[2]);
            aux_put(3, Nb);
        }
        aux_put(4, ds.d0);
        aux_put(5, ds.q);
        aux_put(6, ds.dK);
    }
    block_reduce_store<6, 256, true>(th, -1, P.partials + 6 * blockIdx.x);
}

// seed: the final moment phi_T (Eq. Moment0_Phi) of the state at P.src_base receives
// dL/dphi_T: lambda = 0, c_F = dL/dphi dphi/dF, theta via dphi/dK
template <class SL, class FL, int PREC>
__global__ void __launch_bounds__(256) k_adj_seed(const KParams P, long long nodes,
                                                  const double* __restrict__ dL_dphi) {
    using SLOTS = Slots<FL::Q, SL::Q>;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double th[6] = {0, 0, 0, 0, 0, 0};
    if (i < nodes) {
        const int x = int(i % P.nx), y = int((i / P.nx) % P.ny), z = int(i / ((long long)P.nx * P.ny));
        const Nbr nb = neighbours(x, y, z, P);
        double ps = 0.0, cA = 0.0, cB = 0.0;
        static_for<0, SL::Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            unsigned t;
            const char* sg = pull_src<SLOTS, SL, SLOTS::G0 + k, k>(P.src_base, P, z, unsigned(i), nb, t);
            const char* sa = pull_src<SLOTS, SL, SLOTS::A0 + k, k>(P.src_base, P, z, unsigned(i), nb, t);
            const char* sb = pull_src<SLOTS, SL, SLOTS::B0 + k, k>(P.src_base, P, z, unsigned(i), nb, t);
            ps += double(ld_at<PREC, SLOTS::rest(SLOTS::G0 + k)>(sg, t, float(SL::w(k)) * P.fref[1], P.finv[1]));
            cA += double(ld_at<PREC, SLOTS::rest(SLOTS::A0 + k)>(sa, t, float(SL::w(k)) * P.fref[2], P.finv[2]));
            cB += double(ld_at<PREC, SLOTS::rest(SLOTS::B0 + k)>(sb, t, float(SL::w(k)) * P.fref[3], P.finv[3]));
        });
        const PhiSens ds = phi_sensitivities(ps, cA, cB, P);
        const double s = dL_dphi[i];
        for (int k = 0; k < SLOTS::N; ++k) *adj_at<SL, FL>(P.adj_out, P, k, i) = 0.0f;
        float* c = P.auxc;
        c[0 * P.aux_stride + i] = float(s * ds.d0);
        c[1 * P.aux_stride + i] = float(s * ds.q * (P.c1A - P.c0A));
        c[2 * P.aux_stride + i] = float(s * ds.q * (P.c1B - P.c0B));
        theta_from_K(s * ds.dK, P, th);
    }
    block_reduce_store<6, 256, true>(th, -1, P.partials + 6 * blockIdx.x);
}

// Transpose of the phi stencil (mirror ghosts at walls, wrap otherwise): node y
// collects psi(y) = sum over (x, k) with map(x + e_k) = y of 3 w_k (e_k . Gb(x) + Nb(x)),
// Gb, Nb = aux rows 0..3.  GMODE 0 (adjoint step): phi(y) = Phi(sum g, c^A, c^B)(y), so
// c_F(y) = psi(y) dphi/dF(y) (aux rows 4, 5) and theta receives psi(y) dphi/dK(y)
// (aux row 6).  GMODE 1 (initial state, phi_0 an input): grad_phi0(y) = aux row 4 + psi(y).
template <class SL, class FL, int GMODE>
__global__ void __launch_bounds__(256) k_adj_gather(const KParams P, long long nodes, double* __restrict__ grad_phi0) {
    using STL = typename std::conditional<SL::DIM == 2, D2Q9K, D3Q19K>::type;
    const unsigned i = blockIdx.x * 256u + threadIdx.x;
    double th[6] = {0, 0, 0, 0, 0, 0};
    if (i < (unsigned long long)nodes) {
        const unsigned nxny = unsigned(P.nx) * unsigned(P.ny);
        const int z = int(i / nxny), r = int(i - unsigned(z) * nxny);
        const int y = r / P.nx, x = r - y * P.nx;
        const int yc[3] = {x, y, z};
        const int n[3] = {P.nx, P.ny, P.nz};
        const int wall[3] = {P.wall_x, P.wall_y, P.wall_z};
        const unsigned long long as = P.aux_stride;
        auto row = [&](int rr) { return reinterpret_cast<const char*>(P.aux + (unsigned long long)rr * as); };
        auto at = [&](int rr, unsigned node) { return *reinterpret_cast<const float*>(row(rr) + voff(node * 4u)); };
        float psi = 0.0f;
        if constexpr (FL::Q > 0) {
            bool near_wall = false;
            for (int a = 0; a < 3; ++a) near_wall |= wall[a] && (yc[a] == 0 || yc[a] == n[a] - 1);
            if (!near_wall) {
                // sources x = wrap(y - e_k)
                const Nbr nb = neighbours(x, y, z, P);
                static_for<1, STL::Q>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    constexpr int ex = STL::ex(k), ey = STL::ey(k), ez = STL::ez(k);
                    const unsigned xs = unsigned(int(i) + pull_offset<ex, ey, ez>(nb));
                    float gb = at(3, xs);
                    if constexpr (ex != 0) gb += ex > 0 ? at(0, xs) : -at(0, xs);
                    if constexpr (ey != 0) gb += ey > 0 ? at(1, xs) : -at(1, xs);
                    if constexpr (ez != 0) gb += ez > 0 ? at(2, xs) : -at(2, xs);
                    psi += float(3.0 * STL::w(k)) * gb;
                });
            } else {
                // along a wall axis a source is y - e_k when inside, and y itself when
                // y + e_k lies beyond the wall (its mirror ghost is y)
                static_for<1, STL::Q>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    constexpr int e[3] = {STL::ex(k), STL::ey(k), STL::ez(k)};
                    int cand[3][2], nc[3];
                    for (int a = 0; a < 3; ++a) {
                        nc[a] = 0;
                        if (e[a] == 0) {
                            cand[a][nc[a]++] = yc[a];
                        } else if (!wall[a]) {
                            cand[a][nc[a]++] = (yc[a] - e[a] + n[a]) % n[a];
                        } else {
                            const int sa = yc[a] - e[a];
                            if (sa >= 0 && sa < n[a]) cand[a][nc[a]++] = sa;
                            if ((e[a] < 0 && yc[a] == 0) || (e[a] > 0 && yc[a] == n[a] - 1)) cand[a][nc[a]++] = yc[a];
                        }
                    }
                    for (int i0 = 0; i0 < nc[0]; ++i0)
                        for (int i1 = 0; i1 < nc[1]; ++i1)
                            for (int i2 = 0; i2 < nc[2]; ++i2) {
                                const unsigned xs = unsigned((cand[2][i2] * P.ny + cand[1][i1]) * P.nx + cand[0][i0]);
                                float gb = at(3, xs);
                                if constexpr (e[0] != 0) gb += e[0] * at(0, xs);
                                if constexpr (e[1] != 0) gb += e[1] * at(1, xs);
                                if constexpr (e[2] != 0) gb += e[2] * at(2, xs);
                                psi += float(3.0 * STL::w(k)) * gb;
                            }
                });
            }
        }
        if constexpr (GMODE == 1) {
            grad_phi0[i] = double(at(4, i)) + double(psi);
        } else {
            const float q = at(5, i);
            char* cbase = reinterpret_cast<char*>(P.auxc);
            const unsigned o = voff(i * 4u);
            *reinterpret_cast<float*>(cbase + o) = psi * at(4, i);
            *reinterpret_cast<float*>(cbase + as * 4u + o) = psi * q * float(P.c1A - P.c0A);
            *reinterpret_cast<float*>(cbase + 2 * as * 4u + o) = psi * q * float(P.c1B - P.c0B);
            theta_from_K(double(psi) * double(at(6, i)), P, th);
        }
    }
    if constexpr (GMODE == 0) block_reduce_store<6, 256, true>(th, -1, P.partials + 6 * blockIdx.x);
}

// Adjoint of the initialisation (k_init) with mu_0 held fixed: the adjoint of the
// initial populations (lambda + c in P.adj_in / aux) back to phi_0.  Local part per
// node into aux (rows 0..3: Gb, Nb of the F_0 stencil; row 4: local dL/dphi_0), theta
// partials per work-group; the stencil part closes in k_adj_gather<.., 1>.
template <class SL, class FL>
__global__ void __launch_bounds__(256) k_adj_init_local(const KParams P, long long nodes,
                                                        const double* __restrict__ phi0,
                                                        const double* __restrict__ muA0,
                                                        const double* __restrict__ muB0) {
    using SLOTS = Slots<FL::Q, SL::Q>;
    using STL = typename std::conditional<SL::DIM == 2, D2Q9K, D3Q19K>::type;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double th[6] = {0, 0, 0, 0, 0, 0};
    if (i < nodes) {
        const int x = int(i % P.nx), y = int((i / P.nx) % P.ny), z = int(i / ((long long)P.nx * P.ny));
        const unsigned long long as = P.aux_stride;
        const float* c = P.auxc;
        const double cg = c[0 * as + i], cAa = c[1 * as + i], cBb = c[2 * as + i];
        const double phi = phi0[i], muA = muA0[i], muB = muB0[i];
        const double dA = P.c1A - P.c0A, dB = P.c1B - P.c0B;
        const double K = P.mphi_w2;
        const double dw = muA * dA + muB * dB;
        double phi_b = 0.0, S_b = 0.0;
        // g_k = w_k phi - w_k S_0 / 2; h_0 = c - (1 - w_0) mu, c = mu + c_0 + p(phi)(c_1 - c_0)
        for (int k = 0; k < SL::Q; ++k) {
            const double lg = double(*adj_at<SL, FL>(P.adj_in, P, SLOTS::G0 + k, i)) + cg;
            phi_b += lg * SL::w(k);
            S_b += -0.5 * lg * SL::w(k);
        }
        const double lA = double(*adj_at<SL, FL>(P.adj_in, P, SLOTS::A0, i)) + cAa;
        const double lB = double(*adj_at<SL, FL>(P.adj_in, P, SLOTS::B0, i)) + cBb;
        phi_b += (lA * dA + lB * dB) * interp_dp(phi);
        // S_0 = K (lambda p'(phi) dw - omega_dw'(phi))
        theta_from_K(S_b * (P.lam * interp_dp(phi) * dw - dwell_d(phi)), P, th);
        phi_b += S_b * K * (P.lam * interp_ddp(phi) * dw - dwell_dd(phi));
        double Gb[3] = {0.0, 0.0, 0.0}, Nb = 0.0;
        if constexpr (FL::Q > 0) {
            // f_k = -w_k (e_k . F_0) / 2
            double F_b[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < FL::Q; ++k) {
                const double lf = *adj_at<SL, FL>(P.adj_in, P, k, i);
                F_b[0] += -0.5 * FL::w(k) * FL::ex(k) * lf;
                F_b[1] += -0.5 * FL::w(k) * FL::ey(k) * lf;
                F_b[2] += -0.5 * FL::w(k) * FL::ez(k) * lf;
            }
            double G[3] = {0.0, 0.0, 0.0}, N = 0.0;
            for (int k = 1; k < STL::Q; ++k) {
                const int xn = map_coord(x + STL::ex(k), P.nx, P.wall_x);
                const int yn = map_coord(y + STL::ey(k), P.ny, P.wall_y);
                const int zn = map_coord(z + STL::ez(k), P.nz, P.wall_z);
                const double v = phi0[(zn * P.ny + yn) * P.nx + xn];
                G[0] += 3.0 * STL::w(k) * STL::ex(k) * v;
                G[1] += 3.0 * STL::w(k) * STL::ey(k) * v;
                G[2] += 3.0 * STL::w(k) * STL::ez(k) * v;
                N += 3.0 * STL::w(k) * v;
            }
            const double lap = 2.0 * N - 6.0 * (1.0 - STL::w(0)) * phi;
            const double bracket = P.cap * (dwell_d(phi) * P.inv_W2 - lap);
            phi_b += P.drho * (F_b[0] * P.gx + F_b[1] * P.gy + F_b[2] * P.gz);
            const double bracket_b = F_b[0] * G[0] + F_b[1] * G[1] + F_b[2] * G[2];
            for (int d = 0; d < 3; ++d) Gb[d] = bracket * F_b[d];
            phi_b += bracket_b * P.cap * P.inv_W2 * dwell_dd(phi);
            const double lap_b = -bracket_b * P.cap;
            th[5] += bracket_b * (P.cap / P.W) * (-dwell_d(phi) * P.inv_W2 - lap);
            Nb = 2.0 * lap_b;
            phi_b += -6.0 * (1.0 - STL::w(0)) * lap_b;
        }
        P.aux[0 * as + i] = float(Gb[0]);
        P.aux[1 * as + i] = float(Gb[1]);
        P.aux[2 * as + i] = float(Gb[2]);
        P.aux[3 * as + i] = float(Nb);
        P.aux[4 * as + i] = float(phi_b);
    }
    block_reduce_store<6, 256, true>(th, -1, P.partials + 6 * blockIdx.x);
}

// the adjoint as FP64 [slot][node] (lambda + c_F) from P.adj_in, or from such an
// array into P.adj_out (lambda = value, c_F = 0)
template <class SL, class FL, bool SET>
__global__ void __launch_bounds__(256) k_adj_copy(const KParams P, long long nodes, double* buf) {
    using SLOTS = Slots<FL::Q, SL::Q>;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= nodes || s >= SLOTS::N) return;
    const int F = s < SLOTS::G0 ? -1 : (s - SLOTS::G0) / SL::Q;
    float* c = P.auxc;
    if constexpr (SET) {
        *adj_at<SL, FL>(P.adj_out, P, s, i) = float(buf[s * nodes + i]);
        if (s == 0) {
            for (int f = 0; f < 3; ++f) c[f * P.aux_stride + i] = 0.0f;
        }
    } else {
        double v = *adj_at<SL, FL>(P.adj_in, P, s, i);
        if (F >= 0) v += double(c[F * P.aux_stride + i]);
        buf[s * nodes + i] = v;
    }
}

// zero n doubles
template <int NT = 256>
__global__ void __launch_bounds__(NT) k_zero_f64(double* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// per-work-group sums of a double field (grid-stride, fixed order)
template <int NT = 256>
__global__ void __launch_bounds__(256) k_sum_partials(const double* __restrict__ v, long long n,
                                                      double* __restrict__ partials) {
    double acc[1] = {0.0};
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        acc[0] += v[i];
    block_reduce_store<1, 256>(acc, -1, partials + blockIdx.x);
}

// final fixed-order reduction of per-work-group partials (one work-group).
// partials are [nparts][N]; out[i] = scale[i] * reduce_i(partials[.][i]), except that
// the last entry goes to out[LAST_AT]
template <int N, bool ACC = false, int LAST_AT = N - 1>
__global__ void __launch_bounds__(256) k_finalize(const double* __restrict__ partials, int nparts,
                                                  int maxslot, double scale0, double* __restrict__ out) {
    double acc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = 0.0;
    for (int p = threadIdx.x; p < nparts; p += 256) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double v = partials[p * N + i];
            acc[i] = (i == maxslot) ? fmax(acc[i], v) : acc[i] + v;
        }
    }
    double res[N];
    block_reduce_store<N, 256>(acc, maxslot, res);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double v = (i == 0) ? res[i] * scale0 : res[i];
            const int o = (i == N - 1) ? LAST_AT : i;
            if constexpr (ACC) out[o] += v;
            else out[o] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// droplet count (Section 4.2.2): Euler characteristic chi = sum over the
// elements of the cell complex of (-1)^dim, where the complex is the union of the
// closed unit cells of the nodes whose mask byte is set.  Every element is the
// cell-like part S (a subset of the axes) of one anchor: along the axes in S it is
// the cell interval j, along the others the vertex position between cells j - 1
// and j.  It belongs to the complex when one of the 2^(d - |S|) cells containing
// it is set, and has dimension |S|.  One thread per anchor reads the 2^d cells
// around it (cells across a wall are empty, periodic axes wrap), so every element
// is counted once.  The grid strides over the anchors; partials[blockIdx.x]
// receives the work-group's sum (an integer, exact in FP64).

template <int D>
__global__ void __launch_bounds__(256) k_euler(const unsigned char* __restrict__ mask, const EulerGeom G,
                                               double* __restrict__ partials) {
    int acc = 0;
    const long long step = (long long)gridDim.x * 256;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < G.nanchors; t += step) {
        int j[D];
        long long r = t;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const long long m = G.n[a] + G.wall[a];
            j[a] = int(r % m);
            r /= m;
        }
        // bit o set: cell (j_a - 1 + o_a)_a is in the complex (o_a = bit a of o)
        unsigned bits = 0;
#pragma unroll
        for (int o = 0; o < (1 << D); ++o) {
            long long off = 0;
            bool in = true;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                int c = j[a] - 1 + ((o >> a) & 1);
                if (c < 0) {
                    if (G.wall[a]) in = false;
                    else c += G.n[a];
                } else if (c >= G.n[a]) {
                    if (G.wall[a]) in = false;
                    else c -= G.n[a];
                }
                off += (long long)c * G.stride[a];
            }
            if (in && mask[off]) bits |= 1u << o;
        }
#pragma unroll
        for (int S = 0; S < (1 << D); ++S) {
            bool valid = true;
#pragma unroll
            for (int a = 0; a < D; ++a)
                if (((S >> a) & 1) && j[a] >= G.n[a]) valid = false;  // no cell j past the last one
            // cells containing the element: o has every bit of S
            bool present = false;
#pragma unroll
            for (int o = 0; o < (1 << D); ++o)
                if ((o & S) == S && ((bits >> o) & 1u)) present = true;
            if (valid && present) acc += (__builtin_popcount(S) & 1) ? -1 : 1;
        }
    }
    double v[1] = {double(acc)};
    block_reduce_store<1, 256>(v, -1, partials + blockIdx.x);
}

}  // namespace lbm
