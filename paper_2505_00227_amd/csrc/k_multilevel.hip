// Multilevel decomposition and recomposition of a row-major n0 x n1 x n2 field
// (n2 fastest) into coefficient levels, the input form of Sec. 2/3.  The
// decomposition is prior work that the paper does not spell out; this is the
// hierarchical multilinear interpolation decomposition (MGARD's interpolation
// step without its L2-projection correction).  Step j works on the stride
// h = 2^j grid: a node of it that is not on the stride-2h grid stores
// u - P, where P refines the stride-2h values along x, then y, then z, each
// time taking (a + b) * 0.5 of the two neighbours on the axis, or the left
// neighbour alone past the last coarse node of the line.  Level 0 holds the raw
// values of the stride-2^nsteps grid; level l >= 1 holds the nodes of step
// nsteps - l in the row-major order of their grid.  Arithmetic stays in the
// field's type, one rounding per operation (no contraction), so coefficients
// are reproducible bit for bit.
//
// Decomposition reads only the input field (no node's coefficient depends on
// another's), so one launch covers every level; recomposition needs the
// coarser grid first and runs one launch per step.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mdr_internal.hpp"

namespace mdr {
namespace {

constexpr uint32_t kMl = 256;  // threads per workgroup, along x

__device__ __forceinline__ uint64_t axis_nodes(uint32_t n, uint32_t j)
{
    return n == 0 ? 0 : (uint64_t)((n - 1) >> j) + 1;
}

// position of stride-h node (a, b, c) among its grid's nodes that are not on
// the stride-2h grid, in row-major order (m1, m2: nodes per y / x line)
__device__ __forceinline__ uint64_t new_rank(uint64_t a, uint64_t b, uint64_t c, uint64_t m1, uint64_t m2)
{
    const uint64_t e1 = (m1 + 1) >> 1, e2 = (m2 + 1) >> 1;
    uint64_t skipped = ((a + 1) >> 1) * e1 * e2;  // all-even nodes of earlier planes
    if (!(a & 1)) {
        skipped += ((b + 1) >> 1) * e2;           // ... of earlier rows in this plane
        if (!(b & 1)) skipped += (c + 1) >> 1;    // ... earlier in this row
    }
    return (a * m1 + b) * m2 + c - skipped;
}

struct Axis {
    uint32_t lo, hi;
    bool two;  // mean of lo and hi; otherwise the value at lo
};

__device__ __forceinline__ Axis axis_at(uint32_t i, uint32_t j, uint32_t n)
{
    const uint32_t h = 1u << j;
    if (!((i >> j) & 1u)) return {i, i, false};
    const bool two = i + h < n;
    return {i - h, two ? i + h : i - h, two};
}

// P at node (i0, i1, i2) of step j from the stride-2h values of u
template <typename T>
__device__ __forceinline__ T predict(const T* __restrict__ u, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t i0,
                                     uint32_t i1, uint32_t i2, uint32_t j)
{
#pragma clang fp contract(off)
    const Axis z = axis_at(i0, j, n0), y = axis_at(i1, j, n1), x = axis_at(i2, j, n2);
    const T half = T(0.5);
    auto along_x = [&](uint32_t zz, uint32_t yy) -> T {
        const T* r = u + ((uint64_t)zz * n1 + yy) * n2;
        return x.two ? (r[x.lo] + r[x.hi]) * half : r[x.lo];
    };
    auto along_y = [&](uint32_t zz) -> T {
        return y.two ? (along_x(zz, y.lo) + along_x(zz, y.hi)) * half : along_x(zz, y.lo);
    };
    return z.two ? (along_y(z.lo) + along_y(z.hi)) * half : along_y(z.lo);
}

template <typename T>
__global__ __launch_bounds__(kMl) void k_decompose(const T* __restrict__ u, uint32_t n0, uint32_t n1, uint32_t n2,
                                                   uint32_t nsteps, MlOffsets off, T* __restrict__ out)
{
#pragma clang fp contract(off)
    const uint32_t i2 = blockIdx.x * kMl + threadIdx.x;
    if (i2 >= n2) return;
    const uint32_t i1 = blockIdx.y, i0 = blockIdx.z;
    const uint32_t j = (uint32_t)__builtin_ctz(i0 | i1 | i2 | (1u << nsteps));
    const T v = u[((uint64_t)i0 * n1 + i1) * n2 + i2];
    if (j == nsteps) {
        const uint64_t r = ((uint64_t)(i0 >> j) * axis_nodes(n1, j) + (i1 >> j)) * axis_nodes(n2, j) + (i2 >> j);
        out[off.off[0] + r] = v;
        return;
    }
    const uint64_t r = new_rank(i0 >> j, i1 >> j, i2 >> j, axis_nodes(n1, j), axis_nodes(n2, j));
    out[off.off[nsteps - j] + r] = v - predict(u, n0, n1, n2, i0, i1, i2, j);
}

// coarsest grid: raw values back in place (grid: x blocks, m1, m0 of stride 2^nsteps)
template <typename T>
__global__ __launch_bounds__(kMl) void k_recompose_coarse(const T* __restrict__ c, uint32_t n1, uint32_t n2,
                                                          uint32_t nsteps, T* __restrict__ u)
{
    const uint64_t m2 = axis_nodes(n2, nsteps), m1 = axis_nodes(n1, nsteps);
    const uint32_t b2 = blockIdx.x * kMl + threadIdx.x;
    if (b2 >= m2) return;
    const uint32_t b1 = blockIdx.y, b0 = blockIdx.z;
    const uint64_t idx = ((uint64_t)(b0 << nsteps) * n1 + (b1 << nsteps)) * n2 + (b2 << nsteps);
    u[idx] = c[((uint64_t)b0 * m1 + b1) * m2 + b2];
}

// step j: every stride-h node off the stride-2h grid gets c + P
template <typename T>
__global__ __launch_bounds__(kMl) void k_recompose_step(const T* __restrict__ c, uint32_t n0, uint32_t n1, uint32_t n2,
                                                        uint32_t j, T* __restrict__ u)
{
#pragma clang fp contract(off)
    const uint64_t m2 = axis_nodes(n2, j), m1 = axis_nodes(n1, j);
    const uint32_t b2 = blockIdx.x * kMl + threadIdx.x;
    if (b2 >= m2) return;
    const uint32_t b1 = blockIdx.y, b0 = blockIdx.z;
    if (!((b0 | b1 | b2) & 1u)) return;  // on the coarser grid: already in place
    const uint32_t i0 = b0 << j, i1 = b1 << j, i2 = b2 << j;
    const T p = predict(u, n0, n1, n2, i0, i1, i2, j);
    u[((uint64_t)i0 * n1 + i1) * n2 + i2] = c[new_rank(b0, b1, b2, m1, m2)] + p;
}

dim3 line_grid(uint64_t m0, uint64_t m1, uint64_t m2)
{
    return dim3((uint32_t)((m2 + kMl - 1) / kMl), (uint32_t)m1, (uint32_t)m0);
}

template <typename T>
hipError_t decompose_t(const T* u, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t nsteps, const MlOffsets& off,
                       T* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_decompose<T>, line_grid(n0, n1, n2), dim3(kMl), 0, s, u, n0, n1, n2, nsteps, off, out);
    return hipGetLastError();
}

template <typename T>
hipError_t recompose_t(const T* c, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t nsteps, const MlOffsets& off,
                       T* u, hipStream_t s)
{
    auto m = [&](uint32_t n, uint32_t j) { return n == 0 ? 0ull : (uint64_t)((n - 1) >> j) + 1; };
    hipLaunchKernelGGL(k_recompose_coarse<T>, line_grid(m(n0, nsteps), m(n1, nsteps), m(n2, nsteps)), dim3(kMl), 0,
                       s, c + off.off[0], n1, n2, nsteps, u);
    hipError_t e = hipGetLastError();
    for (uint32_t l = 1; l <= nsteps && e == hipSuccess; ++l) {
        const uint32_t j = nsteps - l;
        hipLaunchKernelGGL(k_recompose_step<T>, line_grid(m(n0, j), m(n1, j), m(n2, j)), dim3(kMl), 0, s,
                           c + off.off[l], n0, n1, n2, j, u);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

hipError_t launch_decompose(bool f64, const void* u, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t nsteps,
                            const MlOffsets& off, void* out, hipStream_t s)
{
    if ((uint64_t)n0 * n1 * n2 == 0) return hipSuccess;
    return f64 ? decompose_t(static_cast<const double*>(u), n0, n1, n2, nsteps, off, static_cast<double*>(out), s)
               : decompose_t(static_cast<const float*>(u), n0, n1, n2, nsteps, off, static_cast<float*>(out), s);
}

hipError_t launch_recompose(bool f64, const void* c, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t nsteps,
                            const MlOffsets& off, void* u, hipStream_t s)
{
    if ((uint64_t)n0 * n1 * n2 == 0) return hipSuccess;
    return f64 ? recompose_t(static_cast<const double*>(c), n0, n1, n2, nsteps, off, static_cast<double*>(u), s)
               : recompose_t(static_cast<const float*>(c), n0, n1, n2, nsteps, off, static_cast<float*>(u), s);
}

}  // namespace mdr
