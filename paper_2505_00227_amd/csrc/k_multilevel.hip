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
// One launch per level.  A decomposition step reads only the input field, so
// its launches are independent; a recomposition step reads the nodes of every
// coarser step, so they run coarsest first.  Within a step a wavefront covers
// part of one row of the step's grid and a lane an (even, odd) pair of its
// nodes (in the finest step, groups of 4): the row's parity, coarse rows and
// output offset are uniform, and consecutive lanes touch consecutive nodes.
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

// The coarse rows a stride-h row (a, b) interpolates from: rows a -/+ 1 when a
// is odd (one of them past the end of the grid), row a itself when it is even;
// the same along y.  Uniform across a workgroup, which covers part of one row.
template <typename T>
struct CoarseRows {
    const T* r[2][2];  // [z side][y side]
    bool z2, y2;       // mean of both sides, else side 0 alone
};

template <typename T>
__device__ __forceinline__ CoarseRows<T> coarse_rows(const T* u, uint32_t n1, uint32_t n2, uint64_t a, uint64_t b,
                                                     uint64_t m0, uint64_t m1, uint32_t j)
{
    CoarseRows<T> cr;
    const uint64_t z0 = (a & 1) ? a - 1 : a, y0 = (b & 1) ? b - 1 : b;
    cr.z2 = (a & 1) && a + 1 < m0;
    cr.y2 = (b & 1) && b + 1 < m1;
    const uint64_t z1 = cr.z2 ? a + 1 : z0, y1 = cr.y2 ? b + 1 : y0;
    auto row = [&](uint64_t zz, uint64_t yy) { return u + ((zz << j) * n1 + (yy << j)) * n2; };
    cr.r[0][0] = row(z0, y0);
    cr.r[0][1] = row(z0, y1);
    cr.r[1][0] = row(z1, y0);
    cr.r[1][1] = row(z1, y1);
    return cr;
}

// P at the pair of stride-h nodes (2t, 2t + 1) of a row: pe for the even node
// (no refinement along x), po for the odd one (mean of coarse nodes 2t and
// 2t + 2, or node 2t alone past the end of the line); then y, then z
template <typename T>
__device__ __forceinline__ void predict_pair(const CoarseRows<T>& cr, uint64_t xe, uint64_t xn, bool x2, T& pe, T& po)
{
#pragma clang fp contract(off)
    const T half = T(0.5);
    T e[2][2], o[2][2];
#pragma unroll
    for (int zi = 0; zi < 2; ++zi)
#pragma unroll
        for (int yi = 0; yi < 2; ++yi) {
            const T* r = cr.r[zi][yi];
            const T v = r[xe];
            e[zi][yi] = v;
            o[zi][yi] = x2 ? (v + r[xn]) * half : v;
        }
    T ey[2], oy[2];
#pragma unroll
    for (int zi = 0; zi < 2; ++zi) {
        ey[zi] = cr.y2 ? (e[zi][0] + e[zi][1]) * half : e[zi][0];
        oy[zi] = cr.y2 ? (o[zi][0] + o[zi][1]) * half : o[zi][0];
    }
    pe = cr.z2 ? (ey[0] + ey[1]) * half : ey[0];
    po = cr.z2 ? (oy[0] + oy[1]) * half : oy[0];
}

// Step j of the decomposition (DEC: field -> level) or of the recomposition
// (field of the coarser steps + level -> field).  Grid: (pairs / kStepX,
// m1 / kStepRows, m0) over the stride-h grid, block (kStepX, kStepRows): a
// wavefront per row (rows of the coarser steps are short), and a lane takes the
// nodes 2t and 2t + 1 of its row.
constexpr uint32_t kStepX = 64, kStepRows = 4;

// In a row with a or b odd every node is new and the row's coefficients are
// contiguous from new_rank(a, b, 0); in a row with both even only odd x is new.
template <typename T, bool DEC>
__device__ __forceinline__ void ml_step_row(const T* __restrict__ in, T* out, const T* field, uint32_t n1,
                                            uint32_t n2, uint32_t j, uint64_t m0, uint64_t a)
{
#pragma clang fp contract(off)
    const uint64_t m1 = axis_nodes(n1, j), m2 = axis_nodes(n2, j);
    const uint64_t t = (uint64_t)blockIdx.x * kStepX + threadIdx.x;
    const uint64_t b = (uint64_t)blockIdx.y * kStepRows + threadIdx.y;
    if (2 * t >= m2 || b >= m1) return;
    const bool coarse_row = !((a | b) & 1);
    const uint64_t base = new_rank(a, b, 0, m1, m2);
    const CoarseRows<T> cr = coarse_rows(field, n1, n2, a, b, m0, m1, j);
    const bool has_odd = 2 * t + 1 < m2;
    const uint64_t xe = (2 * t) << j, xo = (2 * t + 1) << j, xn = (2 * t + 2) << j;
    T pe, po;
    predict_pair(cr, xe, xn, 2 * t + 2 < m2, pe, po);
    const uint64_t self = ((a << j) * n1 + (b << j)) * n2;
    if (DEC) {
        const T* u = in + self;
        if (coarse_row) {
            if (has_odd) out[base + t] = u[xo] - po;
        } else {
            out[base + 2 * t] = u[xe] - pe;
            if (has_odd) out[base + 2 * t + 1] = u[xo] - po;
        }
    } else {
        T* u = out + self;
        if (coarse_row) {
            if (has_odd) u[xo] = in[base + t] + po;
        } else {
            u[xe] = in[base + 2 * t] + pe;
            if (has_odd) u[xo] = in[base + 2 * t + 1] + po;
        }
    }
}

// 16-byte row accesses of 4 consecutive values
__device__ __forceinline__ void load4(const float* p, float o[4])
{
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x, o[1] = v.y, o[2] = v.z, o[3] = v.w;
}
__device__ __forceinline__ void load4(const double* p, double o[4])
{
    const double2 v0 = reinterpret_cast<const double2*>(p)[0], v1 = reinterpret_cast<const double2*>(p)[1];
    o[0] = v0.x, o[1] = v0.y, o[2] = v1.x, o[3] = v1.y;
}
__device__ __forceinline__ void store4(float* p, const float o[4])
{
    *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
}
__device__ __forceinline__ void store4(double* p, const double o[4])
{
    reinterpret_cast<double2*>(p)[0] = make_double2(o[0], o[1]);
    reinterpret_cast<double2*>(p)[1] = make_double2(o[2], o[3]);
}

constexpr uint32_t kFineX = 64, kFineRows = 4;  // workgroup: a wavefront per row, 4 rows

// order LDS traffic between the lanes of one wavefront
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The finest step (j = 0) when rows are whole 16-byte vectors (n2 % 4 == 0,
// 16-byte aligned field): a lane takes kFineG groups of 4 consecutive nodes of
// its row (group g of lane t: nodes 4(g kFineX + t) .. + 3), every load of
// every group issued before any arithmetic so that a wavefront keeps more
// bytes in flight per memory round trip; one 16-byte access per row read per
// group, the same arithmetic as k_ml_step.  The level side (any alignment)
// goes through LDS so that its loads and stores are lane-contiguous: the
// wavefront's coefficients are one contiguous run (4 kFineG kFineX of them, half
// in a row with both indices even, fewer at a row's end).  A wavefront takes
// kFineR rows (b, b + kFineRows, ...), loading all of them first.  Grid:
// (n2 / (4 kFineG kFineX), n1 / (kFineRows kFineR), n0), block (kFineX,
// kFineRows).
constexpr uint32_t kFineG = 2;                      // 4-node groups per lane and row
constexpr uint32_t kFineR = 1;                      // rows per wavefront: b, b + kFineRows, ... (2 was
                                                    // slower: more registers, no more bytes per round trip)
constexpr uint32_t kFineRun = 4 * kFineG * kFineX;  // nodes per wavefront and row

template <typename T, bool DEC>
__device__ __forceinline__ void ml_fine_rows(const T* __restrict__ in, T* out, const T* field, uint32_t n0,
                                             uint32_t n1, uint32_t n2, uint64_t a, T (*w)[kFineRun])
{
#pragma clang fp contract(off)
    const uint32_t lane = threadIdx.x;
    const uint64_t q = n2 / 4;  // groups per row
    const uint64_t g0 = (uint64_t)blockIdx.x * (kFineG * kFineX);
    const uint64_t b0 = (uint64_t)blockIdx.y * (kFineRows * kFineR) + threadIdx.y;
    if (b0 >= n1) return;  // whole wavefront
    const uint64_t wgroups = q - g0 < kFineG * kFineX ? q - g0 : kFineG * kFineX;
    const T half = T(0.5);
    bool rlive[kFineR], coarse_row[kFineR];
    uint64_t wcoef[kFineR], wbase[kFineR], row[kFineR];
    CoarseRows<T> cr[kFineR];
    T v[kFineR][kFineG][2][2][4], nx[kFineR][kFineG][2][2], u[kFineR][kFineG][4];
    bool live[kFineG];
    uint64_t xs[kFineG];
#pragma unroll
    for (uint32_t g = 0; g < kFineG; ++g) {
        const uint64_t grp = g0 + (uint64_t)g * kFineX + lane;  // each access lane-contiguous
        live[g] = grp < q;
        xs[g] = 4 * grp;
    }
    // every load of every row and group first
#pragma unroll
    for (uint32_t rr = 0; rr < kFineR; ++rr) {
        const uint64_t b = b0 + (uint64_t)rr * kFineRows;
        rlive[rr] = b < n1;
        if (!rlive[rr]) continue;
        coarse_row[rr] = !((a | b) & 1);
        wcoef[rr] = coarse_row[rr] ? 2 * wgroups : 4 * wgroups;  // this row's run of coefficients
        wbase[rr] = new_rank(a, b, 0, n1, n2) + (coarse_row[rr] ? 2 : 4) * g0;
        row[rr] = (a * n1 + b) * n2;
        cr[rr] = coarse_rows(field, n1, n2, a, b, n0, n1, 0);
#pragma unroll
        for (uint32_t g = 0; g < kFineG; ++g) {
            if (!live[g]) continue;
#pragma unroll
            for (int zi = 0; zi < 2; ++zi)
#pragma unroll
                for (int yi = 0; yi < 2; ++yi) {
                    const T* r = cr[rr].r[zi][yi];
                    load4(r + xs[g], v[rr][g][zi][yi]);
                    nx[rr][g][zi][yi] = xs[g] + 4 < n2 ? r[xs[g] + 4] : T(0);
                }
            if (DEC) load4(in + row[rr] + xs[g], u[rr][g]);
        }
        if (!DEC) {
#pragma unroll
            for (uint32_t k = 0; k < 4 * kFineG; ++k) {
                const uint64_t i = lane + (uint64_t)k * kFineX;
                if (i < wcoef[rr]) w[rr][i] = in[wbase[rr] + i];
            }
        }
    }
    T c[kFineR][kFineG][4];  // recomposition: coefficients (odd nodes only in a coarse row)
    if (!DEC) {
        wave_sync();
#pragma unroll
        for (uint32_t rr = 0; rr < kFineR; ++rr)
#pragma unroll
            for (uint32_t g = 0; g < kFineG; ++g) {
                const uint32_t slot = g * kFineX + lane;
                if (rlive[rr] && coarse_row[rr]) {
                    c[rr][g][1] = w[rr][2 * slot];
                    c[rr][g][3] = w[rr][2 * slot + 1];
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) c[rr][g][k] = w[rr][4 * slot + k];
                }
            }
        wave_sync();  // every lane has its coefficients before LDS is reused
    }
#pragma unroll
    for (uint32_t rr = 0; rr < kFineR; ++rr) {
        if (!rlive[rr]) continue;
#pragma unroll
        for (uint32_t g = 0; g < kFineG; ++g) {
            if (!live[g]) continue;
            const bool x2 = xs[g] + 4 < n2;  // node x + 3 has a coarse node on its right
            T p[2][2][4];  // per coarse row: P along x of nodes x .. x + 3 (odd ones refined)
#pragma unroll
            for (int zi = 0; zi < 2; ++zi)
#pragma unroll
                for (int yi = 0; yi < 2; ++yi) {
                    const T* vv = v[rr][g][zi][yi];
                    p[zi][yi][0] = vv[0];
                    p[zi][yi][1] = (vv[0] + vv[2]) * half;
                    p[zi][yi][2] = vv[2];
                    p[zi][yi][3] = x2 ? (vv[2] + nx[rr][g][zi][yi]) * half : vv[2];
                }
            T P[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T y0 = cr[rr].y2 ? (p[0][0][k] + p[0][1][k]) * half : p[0][0][k];
                const T y1 = cr[rr].y2 ? (p[1][0][k] + p[1][1][k]) * half : p[1][0][k];
                P[k] = cr[rr].z2 ? (y0 + y1) * half : y0;
            }
            const uint32_t slot = g * kFineX + lane;
            if (DEC) {
                if (coarse_row[rr]) {
                    w[rr][2 * slot] = u[rr][g][1] - P[1];
                    w[rr][2 * slot + 1] = u[rr][g][3] - P[3];
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) w[rr][4 * slot + k] = u[rr][g][k] - P[k];
                }
            } else if (coarse_row[rr]) {
                out[row[rr] + xs[g] + 1] = c[rr][g][1] + P[1];
                out[row[rr] + xs[g] + 3] = c[rr][g][3] + P[3];
            } else {
                T o[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) o[k] = c[rr][g][k] + P[k];
                store4(out + row[rr] + xs[g], o);
            }
        }
    }
    if (DEC) {
        wave_sync();
#pragma unroll
        for (uint32_t rr = 0; rr < kFineR; ++rr) {
            if (!rlive[rr]) continue;
#pragma unroll
            for (uint32_t k = 0; k < 4 * kFineG; ++k) {
                const uint64_t i = lane + (uint64_t)k * kFineX;
                if (i < wcoef[rr]) out[wbase[rr] + i] = w[rr][i];
            }
        }
    }
}

template <typename T, bool DEC>
__global__ __launch_bounds__(kStepX* kStepRows) void k_ml_step(const T* __restrict__ in, T* out, const T* field,
                                                 uint32_t n1, uint32_t n2, uint32_t j, uint64_t m0)
{
    ml_step_row<T, DEC>(in, out, field, n1, n2, j, m0, blockIdx.z);
}

template <typename T, bool DEC>
__global__ __launch_bounds__(kFineX* kFineRows) void k_ml_fine(const T* __restrict__ in, T* out, const T* field,
                                                               uint32_t n0, uint32_t n1, uint32_t n2)
{
    __shared__ T xch[kFineRows][kFineR][kFineRun];
    ml_fine_rows<T, DEC>(in, out, field, n0, n1, n2, blockIdx.z, xch[threadIdx.y]);
}

// coarsest grid (stride 2^nsteps): DEC copies field -> level 0, else back
template <typename T, bool DEC>
__global__ __launch_bounds__(kMl) void k_ml_coarse(const T* __restrict__ in, T* __restrict__ out, uint32_t n1,
                                                   uint32_t n2, uint32_t nsteps)
{
    const uint64_t m2 = axis_nodes(n2, nsteps), m1 = axis_nodes(n1, nsteps);
    const uint64_t b2 = (uint64_t)blockIdx.x * kMl + threadIdx.x;
    if (b2 >= m2) return;
    const uint64_t b1 = blockIdx.y, b0 = blockIdx.z;
    const uint64_t f = ((b0 << nsteps) * n1 + (b1 << nsteps)) * n2 + (b2 << nsteps);
    const uint64_t c = (b0 * m1 + b1) * m2 + b2;
    if (DEC)
        out[c] = in[f];
    else
        out[f] = in[c];
}

dim3 line_grid(uint64_t m0, uint64_t m1, uint64_t m2)
{
    return dim3((uint32_t)((m2 + kMl - 1) / kMl), (uint32_t)m1, (uint32_t)m0);
}

template <typename T>
hipError_t ml_run(bool dec, const T* in, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t nsteps,
                  const MlOffsets& off, T* out, hipStream_t s)
{
    auto m = [&](uint32_t n, uint32_t j) { return n == 0 ? 0ull : (uint64_t)((n - 1) >> j) + 1; };
    const dim3 gc = line_grid(m(n0, nsteps), m(n1, nsteps), m(n2, nsteps));
    if (dec)
        hipLaunchKernelGGL((k_ml_coarse<T, true>), gc, dim3(kMl), 0, s, in, out + off.off[0], n1, n2, nsteps);
    else
        hipLaunchKernelGGL((k_ml_coarse<T, false>), gc, dim3(kMl), 0, s, in + off.off[0], out, n1, n2, nsteps);
    hipError_t e = hipGetLastError();
    // decomposition steps are independent (each reads only the field); the
    // recomposition needs every coarser step first
    const T* field = dec ? in : out;
    const bool fine_vec = n2 % 4 == 0 && reinterpret_cast<uintptr_t>(field) % 16 == 0;
    for (uint32_t l = 1; l <= nsteps && e == hipSuccess; ++l) {
        const uint32_t j = nsteps - l;
        if (j == 0 && fine_vec) {
            const dim3 g((uint32_t)((n2 / 4 + kFineG * kFineX - 1) / (kFineG * kFineX)),
                         (n1 + kFineRows * kFineR - 1) / (kFineRows * kFineR), n0);
            if (dec)
                hipLaunchKernelGGL((k_ml_fine<T, true>), g, dim3(kFineX, kFineRows), 0, s, in, out + off.off[l], in,
                                   n0, n1, n2);
            else
                hipLaunchKernelGGL((k_ml_fine<T, false>), g, dim3(kFineX, kFineRows), 0, s, in + off.off[l], out,
                                   out, n0, n1, n2);
            e = hipGetLastError();
            continue;
        }
        const dim3 g((uint32_t)(((m(n2, j) + 1) / 2 + kStepX - 1) / kStepX),
                     (uint32_t)((m(n1, j) + kStepRows - 1) / kStepRows), (uint32_t)m(n0, j));
        if (dec)
            hipLaunchKernelGGL((k_ml_step<T, true>), g, dim3(kStepX, kStepRows), 0, s, in, out + off.off[l], in, n1,
                               n2, j, m(n0, j));
        else
            hipLaunchKernelGGL((k_ml_step<T, false>), g, dim3(kStepX, kStepRows), 0, s, in + off.off[l], out, out,
                               n1, n2, j, m(n0, j));
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

hipError_t launch_decompose(bool f64, const void* u, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t nsteps,
                            const MlOffsets& off, void* out, hipStream_t s)
{
    if ((uint64_t)n0 * n1 * n2 == 0) return hipSuccess;
    return f64 ? ml_run(true, static_cast<const double*>(u), n0, n1, n2, nsteps, off, static_cast<double*>(out), s)
               : ml_run(true, static_cast<const float*>(u), n0, n1, n2, nsteps, off, static_cast<float*>(out), s);
}

hipError_t launch_recompose(bool f64, const void* c, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t nsteps,
                            const MlOffsets& off, void* u, hipStream_t s)
{
    if ((uint64_t)n0 * n1 * n2 == 0) return hipSuccess;
    return f64 ? ml_run(false, static_cast<const double*>(c), n0, n1, n2, nsteps, off, static_cast<double*>(u), s)
               : ml_run(false, static_cast<const float*>(c), n0, n1, n2, nsteps, off, static_cast<float*>(u), s);
}

}  // namespace mdr
