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

}  // namespace lbm
