// Velocity sets in the kernel frame.
//
// 3D problems use the paper's frame directly.  2D problems run in the x-z
// plane of the kernel frame (ny = 1): the user's y axis is the kernel's z axis,
// so one kernel marches along z in both cases.  The direction order is the
// paper's (Tables tab:D2Q9 and tab:D3Q19); the scalar lattices D2Q5 (0, +x,
// +y, -x, -y) and D3Q7 (0, +x, -x, +y, -y, +z, -z) carry the isotropic
// weights 1/3, 1/6 and 1/4, 1/8 (c_s^2 = 1/3 and 1/4).
#pragma once

#include <type_traits>

namespace lbm {

// compile-time loop: f(std::integral_constant<int, k>) for k in [B, E)
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <int V>
using IC = std::integral_constant<int, V>;

// e . v for a lattice vector with components in {-1, 0, 1}, without the zero terms
template <int EX, int EY, int EZ, class C>
__device__ __forceinline__ C edot(C a, C b, C c) {
    C r = C(0);
    if constexpr (EX != 0) r = EX > 0 ? a : -a;
    if constexpr (EY != 0) {
        if constexpr (EX != 0) r += EY > 0 ? b : -b;
        else r = EY > 0 ? b : -b;
    }
    if constexpr (EZ != 0) {
        if constexpr (EX != 0 || EY != 0) r += EZ > 0 ? c : -c;
        else r = EZ > 0 ? c : -c;
    }
    return r;
}


struct NoLattice {
    static constexpr int Q = 0;
    static constexpr int DIM = 0;
    __host__ __device__ static constexpr int ex(int) { return 0; }
    __host__ __device__ static constexpr int ey(int) { return 0; }
    __host__ __device__ static constexpr int ez(int) { return 0; }
    __host__ __device__ static constexpr int opp(int) { return 0; }
    __host__ __device__ static constexpr double w(int) { return 0.0; }
    static constexpr double cs2 = 1.0;
};

struct D2Q9K {
    static constexpr int Q = 9;
    static constexpr int DIM = 2;
    __host__ __device__ static constexpr int ex(int k) {
        constexpr int a[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        return a[k];
    }
    __host__ __device__ static constexpr int ey(int) { return 0; }
    __host__ __device__ static constexpr int ez(int k) {
        constexpr int a[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        return a[k];
    }
    __host__ __device__ static constexpr int opp(int k) {
        constexpr int a[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
        return a[k];
    }
    __host__ __device__ static constexpr double w(int k) {
        return k == 0 ? 4.0 / 9.0 : (k < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    static constexpr double cs2 = 1.0 / 3.0;
};

struct D3Q19K {
    static constexpr int Q = 19;
    static constexpr int DIM = 3;
    __host__ __device__ static constexpr int ex(int k) {
        constexpr int a[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0};
        return a[k];
    }
    __host__ __device__ static constexpr int ey(int k) {
        constexpr int a[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 1, -1};
        return a[k];
    }
    __host__ __device__ static constexpr int ez(int k) {
        constexpr int a[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 1, -1, 1};
        return a[k];
    }
    __host__ __device__ static constexpr int opp(int k) {
        constexpr int a[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
        return a[k];
    }
    __host__ __device__ static constexpr double w(int k) {
        return k == 0 ? 1.0 / 3.0 : (k < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    static constexpr double cs2 = 1.0 / 3.0;
};

struct D2Q5K {
    static constexpr int Q = 5;
    static constexpr int DIM = 2;
    __host__ __device__ static constexpr int ex(int k) {
        constexpr int a[5] = {0, 1, 0, -1, 0};
        return a[k];
    }
    __host__ __device__ static constexpr int ey(int) { return 0; }
    __host__ __device__ static constexpr int ez(int k) {
        constexpr int a[5] = {0, 0, 1, 0, -1};
        return a[k];
    }
    __host__ __device__ static constexpr int opp(int k) {
        constexpr int a[5] = {0, 3, 4, 1, 2};
        return a[k];
    }
    __host__ __device__ static constexpr double w(int k) { return k == 0 ? 1.0 / 3.0 : 1.0 / 6.0; }
    static constexpr double cs2 = 1.0 / 3.0;
};

struct D3Q7K {
    static constexpr int Q = 7;
    static constexpr int DIM = 3;
    __host__ __device__ static constexpr int ex(int k) {
        constexpr int a[7] = {0, 1, -1, 0, 0, 0, 0};
        return a[k];
    }
    __host__ __device__ static constexpr int ey(int k) {
        constexpr int a[7] = {0, 0, 0, 1, -1, 0, 0};
        return a[k];
    }
    __host__ __device__ static constexpr int ez(int k) {
        constexpr int a[7] = {0, 0, 0, 0, 0, 1, -1};
        return a[k];
    }
    __host__ __device__ static constexpr int opp(int k) {
        constexpr int a[7] = {0, 2, 1, 4, 3, 6, 5};
        return a[k];
    }
    __host__ __device__ static constexpr double w(int k) { return k == 0 ? 0.25 : 0.125; }
    static constexpr double cs2 = 0.25;
};

// ---------------------------------------------------------------------------
// Moment basis of a lattice for the multiple-relaxation-time collision: rows
// orthogonal in the weighted product <a, b> = sum_k w_k a_k b_k, from Gram-Schmidt
// over polynomials in the lattice vector of increasing order (the second order split
// into its trace and traceless parts), skipping those dependent on the lattice.
// The inverse is M^-1_{k i} = w_k M_ik / <M_i, M_i>.  Built at compile time.

template <int Q>
struct MomentBasis {
    double M[Q][Q];
    double invD[Q];  // 1 / <M_i, M_i>
    int order[Q];
};

// value of polynomial j (and its order) at the vector (x, y, z) in 2D or 3D
constexpr double basis_poly(int dim, int j, int x, int y, int z, int& order) {
    if (dim == 2) {
        // 1, x, y, x^2 + y^2, x^2 - y^2, xy, x^2 y, x y^2, x^2 y^2
        const int ord[9] = {0, 1, 1, 2, 2, 2, 3, 3, 4};
        order = ord[j];
        switch (j) {
            case 0: return 1;
            case 1: return x;
            case 2: return y;
            case 3: return x * x + y * y;
            case 4: return x * x - y * y;
            case 5: return x * y;
            case 6: return x * x * y;
            case 7: return x * y * y;
            default: return x * x * y * y;
        }
    }
    const int ord[19] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 4, 4, 4};
    order = ord[j];
    switch (j) {
        case 0: return 1;
        case 1: return x;
        case 2: return y;
        case 3: return z;
        case 4: return x * x + y * y + z * z;
        case 5: return 2 * x * x - y * y - z * z;
        case 6: return y * y - z * z;
        case 7: return x * y;
        case 8: return x * z;
        case 9: return y * z;
        case 10: return x * x * y;
        case 11: return x * x * z;
        case 12: return y * y * x;
        case 13: return y * y * z;
        case 14: return z * z * x;
        case 15: return z * z * y;
        case 16: return x * x * y * y;
        case 17: return x * x * z * z;
        default: return y * y * z * z;
    }
}

// L: a lattice in the kernel frame (2D lattices use x and z)
template <class L>
constexpr MomentBasis<L::Q> make_moment_basis() {
    MomentBasis<L::Q> B{};
    constexpr int Q = L::Q;
    const int npoly = L::DIM == 2 ? 9 : 19;
    int nrows = 0;
    for (int j = 0; j < npoly && nrows < Q; ++j) {
        double v[Q] = {};
        int ord = 0;
        for (int k = 0; k < Q; ++k) {
            // 2D kernel frame: the second axis of the lattice is z
            const int x = L::ex(k), y = L::DIM == 2 ? L::ez(k) : L::ey(k), z = L::DIM == 2 ? 0 : L::ez(k);
            v[k] = basis_poly(L::DIM, j, x, y, z, ord);
        }
        for (int r = 0; r < nrows; ++r) {
            double num = 0, den = 0;
            for (int k = 0; k < Q; ++k) {
                num += L::w(k) * v[k] * B.M[r][k];
                den += L::w(k) * B.M[r][k] * B.M[r][k];
            }
            for (int k = 0; k < Q; ++k) v[k] -= num / den * B.M[r][k];
        }
        double nn = 0;
        for (int k = 0; k < Q; ++k) nn += L::w(k) * v[k] * v[k];
        if (nn > 1e-12) {
            for (int k = 0; k < Q; ++k) B.M[nrows][k] = (v[k] > -1e-12 && v[k] < 1e-12) ? 0.0 : v[k];
            B.invD[nrows] = 1.0 / nn;
            B.order[nrows] = ord;
            ++nrows;
        }
    }
    return B;
}

}  // namespace lbm
