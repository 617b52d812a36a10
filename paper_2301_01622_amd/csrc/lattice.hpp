// Device-side velocity sets for the MI355X kernels.
//
// D3Q27 is the full 3x3x3 cube {-1,0,1}^3 with tensor-product weights
// (2/3 for a zero component, 1/6 for +-1, per axis).  D3Q19 drops the eight
// corners; its weights are 1/3, 1/18, 1/36 by |c|^2.  Both have c_s^2 = 1/3.
// Directions are numbered by their cube index (cx+1) + 3(cy+1) + 9(cz+1),
// D3Q19 keeping the cube order without the corners, so every quantity below
// is a constexpr function of the direction number and folds away in
// unrolled loops.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

template <int Q>
struct Lattice;

namespace detail {
// Cube index of D3Q19 direction i (cube order with the corners removed).
__host__ __device__ constexpr int d3q19_cube(int i)
{
    constexpr int tbl[19] = {1, 3, 4, 5, 7, 9, 10, 11, 12, 13, 14, 15, 16, 17, 19, 21, 22, 23, 25};
    return tbl[i];
}
} // namespace detail

template <>
struct Lattice<27> {
    static constexpr int Q = 27;
    __host__ __device__ static constexpr int cube(int i) { return i; }
    __host__ __device__ static constexpr int cx(int i) { return cube(i) % 3 - 1; }
    __host__ __device__ static constexpr int cy(int i) { return (cube(i) / 3) % 3 - 1; }
    __host__ __device__ static constexpr int cz(int i) { return cube(i) / 9 - 1; }
    __host__ __device__ static constexpr double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
    __host__ __device__ static constexpr double w(int i) { return w1(cx(i)) * w1(cy(i)) * w1(cz(i)); }
};

template <>
struct Lattice<19> {
    static constexpr int Q = 19;
    __host__ __device__ static constexpr int cube(int i) { return detail::d3q19_cube(i); }
    __host__ __device__ static constexpr int cx(int i) { return cube(i) % 3 - 1; }
    __host__ __device__ static constexpr int cy(int i) { return (cube(i) / 3) % 3 - 1; }
    __host__ __device__ static constexpr int cz(int i) { return cube(i) / 9 - 1; }
    __host__ __device__ static constexpr double w(int i)
    {
        return (cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i)) == 0   ? 1.0 / 3.0
               : (cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i)) == 1 ? 1.0 / 18.0
                                                                      : 1.0 / 36.0;
    }
};

// Direction number of -c_i.
template <int Q>
__host__ __device__ constexpr int opposite(int i)
{
    for (int k = 0; k < Q; ++k)
        if (Lattice<Q>::cx(k) == -Lattice<Q>::cx(i) && Lattice<Q>::cy(k) == -Lattice<Q>::cy(i) &&
            Lattice<Q>::cz(k) == -Lattice<Q>::cz(i))
            return k;
    return -1;
}

} // namespace lbm
