// Retrieve kernels for gfx950: bitplane decoding (inverse of Alg. 1) and the
// exact reconstruction of each value from the sign plane and its first k
// magnitude planes.
#include <type_traits>

#include "device_bits.hpp"
#include "mdr_internal.hpp"

namespace mdr {
namespace {

// One thread per block of 32 values: load the sign word and the words of the
// first k planes (plane p holds bit B-1-p), transpose back to magnitudes, and
// write x = (-1)^s * mag * 2^(e-B).  The magnitude keeps at most the input
// type's significand bits, so the integer-to-float conversion and the ldexp
// are exact (subnormal results included).
// One launch covers many levels (of many variables): workgroup -> job via wg_job.
// NT: streaming loads of the plane rows and stores of the f64 output (each is
// touched once); chosen for launches that read most of their planes, while a
// launch of a few planes per level runs with ordinary loads (with streaming
// ones a single 256 MiB level's retrieval at 1e-2 took 0.167 instead of 0.150
// ms, every plane 0.211 instead of 0.240)
template <bool F64, bool NT>
__global__ __launch_bounds__(kThreads) void k_reconstruct(const ReconJob* __restrict__ jobs,
                                                          const uint32_t* __restrict__ wg_job)
{
    using T = std::conditional_t<F64, double, float>;
    // the job's row pointers, staged once per workgroup (uniform LDS reads
    // afterwards instead of one dependent scalar load per row)
    __shared__ const uint32_t* s_rows[kMaxRows];
    const ReconJob& j = jobs[wg_job[blockIdx.x]];
    if (threadIdx.x < kMaxRows) s_rows[threadIdx.x] = j.rows[threadIdx.x];
    const uint32_t nbd = j.nbd, B = j.B, k = j.k, vec = j.vec;
    const uint64_t n = j.n;
    const int e = j.e;
    __syncthreads();
    const uint32_t blk = (blockIdx.x - j.wg_base) * kThreads + threadIdx.x;
    if (blk >= nbd) return;
    const uint64_t base = (uint64_t)blk * 32;
    if (base >= n) return;
    const uint32_t cnt = (uint32_t)min<uint64_t>(32, n - base);
    T* outg = static_cast<T*>(j.out) + base;
    const auto out = gmem(outg);
    T v[32];
    if (k == 0) {
#pragma unroll
        for (int t = 0; t < 32; ++t) v[t] = T(0);
    } else {
        const auto load = [](const uint32_t* row, uint32_t i) -> uint32_t {
            if constexpr (NT)
                return __builtin_nontemporal_load(&gmem(row)[i]);
            else
                return gmem(row)[i];
        };
        const uint32_t sgn = load(s_rows[0], blk);
        uint32_t lo[32];
        uint32_t hi[F64 ? 32 : 1];
        // bit c lives in plane p = B-1-c, present when p < k, i.e. c >= B-k
        // (uniform per workgroup: a branch per row, the held rows' loads all
        // in flight at once; rows that are not held are not read)
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            const bool held = c < (int)B && c >= (int)(B - k);
            lo[c] = held ? load(s_rows[B - c], blk) : 0u;
        }
        transpose32(lo);
        if constexpr (F64) {
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                const bool held = 32 + c < (int)B && 32 + c >= (int)(B - k);
                hi[c] = held ? load(s_rows[B - 32 - c], blk) : 0u;
            }
            transpose32(hi);
        }
        const int sh = e - (int)B;
#pragma unroll
        for (int t = 0; t < 32; ++t) {
            T mag;
            if constexpr (F64)
                mag = (double)hi[t] * 0x1p32 + (double)lo[t];
            else
                mag = (float)lo[t];
            T a = F64 ? (T)__builtin_amdgcn_ldexp((double)mag, sh)
                      : (T)__builtin_amdgcn_ldexpf((float)mag, sh);
            v[t] = ((sgn >> t) & 1u) ? -a : a;
        }
    }
    if constexpr (!F64) {
        // a workgroup of full blocks writes its 8192 consecutive values through
        // LDS, so that every store instruction covers 1 KiB of contiguous output
        // (rows padded to 33 values: conflict-free on both sides)
        __shared__ float s_out[kThreads * 33];
        const uint32_t wblk0 = (blockIdx.x - j.wg_base) * kThreads;
        if (vec && (uint64_t)(wblk0 + kThreads) * 32 <= n) {  // uniform; no thread returned early
#pragma unroll
            for (int t = 0; t < 32; ++t) s_out[threadIdx.x * 33 + t] = v[t];
            __syncthreads();
            const auto p = gmem(reinterpret_cast<f32x4*>(static_cast<float*>(j.out) + (uint64_t)wblk0 * 32));
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t i4 = q * kThreads + threadIdx.x;  // 16-byte slot of the workgroup's output
                const uint32_t b = i4 >> 3, t = (i4 & 7) * 4;     // its block and first value
                p[i4] = f32x4{s_out[b * 33 + t], s_out[b * 33 + t + 1], s_out[b * 33 + t + 2], s_out[b * 33 + t + 3]};
            }
            return;
        }
    }
    if constexpr (F64) {
        // a wavefront of full blocks writes its 2048 consecutive values through
        // LDS in two halves: each store instruction then fills eight whole
        // 128-byte lines (half a block each) instead of a 16-byte piece of 64
        // lines (rows padded to 17 values)
        __shared__ double s_o64[kThreads / 64][64 * 17];
        const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const uint64_t wblk0 = (uint64_t)(blockIdx.x - j.wg_base) * kThreads + wave * 64;
        // uniform per wavefront: every block of it is full (none returned early)
        if (vec && (wblk0 + 64) * 32 <= n) {
            double* so = s_o64[wave];
            const auto p = gmem(reinterpret_cast<f64x2*>(static_cast<double*>(j.out) + wblk0 * 32));
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int t = 0; t < 16; ++t) so[lane * 17 + t] = v[16 * h + t];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint32_t i2 = q * 64 + lane;            // 16-byte slot of the half
                    const uint32_t b = i2 >> 3, t = (i2 & 7) * 2;  // its block and first value
                    const f64x2 pair = f64x2{so[b * 17 + t], so[b * 17 + t + 1]};
                    if constexpr (NT)
                        __builtin_nontemporal_store(pair, &p[b * 16 + h * 8 + (i2 & 7)]);
                    else
                        p[b * 16 + h * 8 + (i2 & 7)] = pair;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            return;
        }
    }
    if (vec && cnt == 32) {
        if constexpr (F64) {
            const auto p = gmem(reinterpret_cast<f64x2*>(outg));
#pragma unroll
            for (int q = 0; q < 16; ++q) p[q] = f64x2{v[2 * q], v[2 * q + 1]};
        } else {
            const auto p = gmem(reinterpret_cast<f32x4*>(outg));
#pragma unroll
            for (int q = 0; q < 8; ++q) p[q] = f32x4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
        }
    } else {
#pragma unroll
        for (int t = 0; t < 32; ++t)
            if ((uint32_t)t < cnt) out[t] = v[t];
    }
}

// QoI error estimates (Sec. 5.2).  With |v_c - vhat_c| <= eps_c per variable,
// each family's score at a point, evaluated in double in this order (no
// contraction: the library is built with -ffp-contract=off):
//   sum of squares (V_total for three variables): D = sum_c eps_c (2|vhat_c| + eps_c),
//     since |v^2 - vhat^2| <= eps (2|vhat| + eps);
//   magnitude sqrt(sum v_c^2): D^2 / Shat, Shat = (vx^2 + vy^2) + vz^2 (+inf
//     when Shat = 0), since |M - Mhat| <= |S - Shat| / Mhat; the host takes
//     the root of its minimum with sum eps_c^2 (the norm of the error vector);
//   product v_0 v_1: (|vhat_0| eps_1 + |vhat_1| eps_0) + eps_0 eps_1.
// Absent variables have zero bounds (their terms are exact zeros); the
// magnitude also leaves them out of Shat.  Many (request, level) jobs in one
// launch; each job folds its maximum into its own accumulator.
template <bool F64>
__device__ __forceinline__ double qoi_score(const QoiJob& j, double vx, double vy, double vz)
{
    const double ex = j.eps[0], ey = j.eps[1], ez = j.eps[2];
    const double ax = fabs(vx), ay = fabs(vy), az = fabs(vz);
    if (j.kind == kQoiProduct) {
        double r = (ax * ey) + (ay * ex);
        return r + (ex * ey);
    }
    double s = 0.0;
    s = s + ex * ((2.0 * ax) + ex);
    s = s + ey * ((2.0 * ay) + ey);
    s = s + ez * ((2.0 * az) + ez);
    if (j.kind == kQoiSumsq) return s;
    double sh = vx * vx;
    if (j.nvars > 1) sh = sh + (vy * vy);
    if (j.nvars > 2) sh = sh + (vz * vz);
    return sh == 0.0 ? __builtin_huge_val() : (s * s) / sh;
}

// Points of a job in vectors of 16 bytes (4 f32 or 2 f64 values of each
// variable), two vectors in flight per thread, then the scalar tail; a
// variable the family does not use is not read (its bound is 0, its term an
// exact zero).  F(value index, vx, vy, vz) is called once per point, in index
// order within each thread.
template <bool F64, class F>
__device__ __forceinline__ void qoi_points(const QoiJob& j, F&& f)
{
    using T = std::conditional_t<F64, double, float>;
    using V = std::conditional_t<F64, f64x2, f32x4>;
    constexpr uint32_t P = 16 / sizeof(T);
    const auto x = gmem(static_cast<const T*>(j.x));
    const auto y = gmem(static_cast<const T*>(j.y));
    const auto z = gmem(static_cast<const T*>(j.z));
    const bool use_y = j.nvars > 1, use_z = j.nvars > 2;
    const uint64_t t0 = (uint64_t)(blockIdx.x - j.wg_base) * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)j.grid * blockDim.x;
    uint64_t done = 0;  // points covered by whole vectors
    if (j.vec) {
        const uint64_t nv = j.n / P;
        const auto xv = gmem(reinterpret_cast<const V*>(static_cast<const T*>(j.x)));
        const auto yv = gmem(reinterpret_cast<const V*>(static_cast<const T*>(j.y)));
        const auto zv = gmem(reinterpret_cast<const V*>(static_cast<const T*>(j.z)));
        const V zero{};
        for (uint64_t v = t0; v < nv; v += 2 * stride) {
            const uint64_t w = v + stride;
            const bool two = w < nv;
            const V ax = xv[v], ay = use_y ? yv[v] : zero, az = use_z ? zv[v] : zero;
            const V bx = two ? xv[w] : zero, by = two && use_y ? yv[w] : zero, bz = two && use_z ? zv[w] : zero;
#pragma unroll
            for (uint32_t q = 0; q < P; ++q) f(v * P + q, (double)ax[q], (double)ay[q], (double)az[q]);
            if (two) {
#pragma unroll
                for (uint32_t q = 0; q < P; ++q) f(w * P + q, (double)bx[q], (double)by[q], (double)bz[q]);
            }
        }
        done = nv * P;
    }
    for (uint64_t i = done + t0; i < j.n; i += stride)
        f(i, (double)x[i], use_y ? (double)y[i] : 0.0, use_z ? (double)z[i] : 0.0);
}

template <bool F64>
__global__ __launch_bounds__(kThreads) void k_qoi_batch(const QoiJob* __restrict__ jobs,
                                                        const uint32_t* __restrict__ wg_job)
{
    const QoiJob& j = jobs[wg_job[blockIdx.x]];
    double worst = 0.0;
    qoi_points<F64>(j, [&](uint64_t, double vx, double vy, double vz) {
        const double sc = qoi_score<F64>(j, vx, vy, vz);
        worst = sc > worst ? sc : worst;
    });
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double o = __shfl_xor(worst, off, 64);
        worst = o > worst ? o : worst;
    }
    __shared__ double s_w[kThreads / 64];
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = worst;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) worst = s_w[w] > worst ? s_w[w] : worst;
        atomicMax(j.acc, (unsigned long long)__double_as_longlong(worst));
    }
}

// The point the CP estimator works on: the smallest index whose score,
// evaluated exactly as above, has the bit pattern of the maximum the previous
// launch left in *acc.
template <bool F64>
__global__ __launch_bounds__(kThreads) void k_qoi_argmax_batch(const QoiJob* __restrict__ jobs,
                                                               const uint32_t* __restrict__ wg_job)
{
    const QoiJob& j = jobs[wg_job[blockIdx.x]];
    const unsigned long long target = *j.acc;
    unsigned long long first = ~0ull;
    qoi_points<F64>(j, [&](uint64_t i, double vx, double vy, double vz) {
        const double sc = qoi_score<F64>(j, vx, vy, vz);
        const unsigned long long at = j.base + i;
        if ((unsigned long long)__double_as_longlong(sc) == target && at < first) first = at;
    });
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(first, off, 64);
        first = o < first ? o : first;
    }
    if ((threadIdx.x & 63) == 0 && first != ~0ull) atomicMin(j.arg, first);
}

// Device values into pinned host memory: every thread of the grid walks all
// spans with one stride, so each span's words go out as consecutive 256-byte
// wavefront stores; system-scope stores write through to host memory.  Runs
// on its own stream beside the compute.
__global__ __launch_bounds__(kThreads) void k_copy_out(const CopySpans sp)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t k = 0; k < sp.n; ++k) {
        const uint32_t* src = sp.src[k];
        uint32_t* dst = sp.dst[k];
        const uint64_t nw = sp.words[k];
        for (uint64_t i = t; i < nw; i += stride)
            __hip_atomic_store(dst + i, src[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace

hipError_t launch_copy_out(const CopySpans& sp, hipStream_t s)
{
    if (sp.n == 0) return hipSuccess;
    if (sp.n > kCopySpans) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy_out, dim3(2048), dim3(kThreads), 0, s, sp);
    return hipGetLastError();
}

hipError_t launch_qoi_vtotal_argmax_batch(const QoiJob* jobs, const uint32_t* wg_job, uint32_t grid, bool f64,
                                          hipStream_t s)
{
    if (grid == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL((k_qoi_argmax_batch<true>), dim3(grid), dim3(kThreads), 0, s, jobs, wg_job);
    else
        hipLaunchKernelGGL((k_qoi_argmax_batch<false>), dim3(grid), dim3(kThreads), 0, s, jobs, wg_job);
    return hipGetLastError();
}

hipError_t launch_qoi_vtotal_batch(const QoiJob* jobs, const uint32_t* wg_job, uint32_t grid, bool f64,
                                   hipStream_t s)
{
    if (grid == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL((k_qoi_batch<true>), dim3(grid), dim3(kThreads), 0, s, jobs, wg_job);
    else
        hipLaunchKernelGGL((k_qoi_batch<false>), dim3(grid), dim3(kThreads), 0, s, jobs, wg_job);
    return hipGetLastError();
}

hipError_t launch_reconstruct_batch(const ReconJob* jobs, const uint32_t* wg_job, uint32_t grid,
                                   bool f64, bool streaming, hipStream_t s)
{
    if (grid == 0) return hipSuccess;
    if (f64 && streaming)
        hipLaunchKernelGGL((k_reconstruct<true, true>), dim3(grid), dim3(kThreads), 0, s, jobs, wg_job);
    else if (f64)
        hipLaunchKernelGGL((k_reconstruct<true, false>), dim3(grid), dim3(kThreads), 0, s, jobs, wg_job);
    else if (streaming)
        hipLaunchKernelGGL((k_reconstruct<false, true>), dim3(grid), dim3(kThreads), 0, s, jobs, wg_job);
    else
        hipLaunchKernelGGL((k_reconstruct<false, false>), dim3(grid), dim3(kThreads), 0, s, jobs, wg_job);
    return hipGetLastError();
}

}  // namespace mdr
