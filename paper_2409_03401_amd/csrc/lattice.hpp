// Velocity sets in the kernel frame.
//
// 3D problems use the paper's frame directly.  2D problems run in the x-z
// plane of the kernel frame (ny = 1): the user's y axis is the kernel's z axis,
// so one kernel marches along z in both cases.  The direction order is the
// paper's (Tables tab:D2Q9 and tab:D3Q19); the scalar lattices D2Q5 (0, +x,
// +y, -x, -y) and D3Q7 (0, +x, -x, +y, -y, +z, -z) carry the isotropic
// weights 1/3, 1/6 and 1/4, 1/8 (c_s^2 = 1/3 and 1/4).
#pragma once

namespace lbm {

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
