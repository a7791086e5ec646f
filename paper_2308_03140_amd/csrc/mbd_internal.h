// Internal definitions shared by the HIP kernels and the host runtime of
// libmbd_hip.so.  Not part of the public C ABI (see include/mbd.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#define MBD_TILE 64          // SYMV / assembly tile edge (rows of one wavefront)
#define MBD_THREADS 256      // 4 wavefronts of 64 lanes

// Error codes mirrored from include/mbd.h
#define MBD_OK_ 0
#define MBD_ERR_INVALID_ARGUMENT_ 1
#define MBD_ERR_NEGATIVE_EIGENVALUE_ 2
#define MBD_ERR_NOT_CONVERGED_ 3
#define MBD_ERR_OUT_OF_MEMORY_ 4
#define MBD_ERR_DEVICE_ 5
#define MBD_ERR_UNSUPPORTED_ 6

// Device status word bits (written by kernels, read once at the end of a call)
#define MBD_ST_BAD_INPUT 1u        // non-finite or non-positive per-atom input
#define MBD_ST_COINCIDENT 2u       // two atoms closer than 1e-8 bohr
#define MBD_ST_COLLAPSE 4u         // some eigenvalue of Q <= 0

static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
static inline long long ceil_div_ll(long long a, long long b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Wavefront / block reductions (deterministic: fixed butterfly then lane-0
// broadcast, so every lane sees bit-identical values)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return __shfl(v, 0, 64);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return __shfl(v, 0, 64);
}

// Sum over a 256-thread block; result valid in every thread.  `red` must hold
// 4 elements of LDS.
template <typename T>
__device__ __forceinline__ T block_sum256(T v, T* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    T r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

template <typename T>
__device__ __forceinline__ T block_max256(T v, T* red) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    T r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Raw buffer loads (gfx9 descriptor, stride 0).  A byte offset at or beyond
// num_records reads as zero, so masked elements are fetched without a branch
// by giving them the offset OOB_OFFSET.
// ---------------------------------------------------------------------------
#define OOB_OFFSET 0x80000000u
// The descriptor must be wave-uniform: base and size are passed through
// readfirstlane so the compiler keeps it in scalar registers (a descriptor it
// cannot prove uniform is wrapped in a per-load waterfall loop).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes) {
    const unsigned long long a = (unsigned long long)base;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    const unsigned nb = __builtin_amdgcn_readfirstlane(bytes);
    return __builtin_amdgcn_make_buffer_rsrc((void*)(((unsigned long long)hi << 32) | lo), (short)0, (int)nb,
                                             0x00020000);
}
template <typename T> __device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <> __device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// 16 bytes per lane: 4 floats or 2 doubles (offset a multiple of 16)
template <typename T> struct Vec16 { typedef T v __attribute__((ext_vector_type(16 / sizeof(T)))); };
template <typename T>
__device__ __forceinline__ typename Vec16<T>::v buf_load16(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(typename Vec16<T>::v, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

template <typename T> struct num_limits;
template <> struct num_limits<double> { static constexpr double eps = 2.220446049250313e-16; };
template <> struct num_limits<float> { static constexpr float eps = 1.1920929e-07f; };

// ---------------------------------------------------------------------------
// Batched dense storage: matrix b of a batch lives at base + b*stride, column
// major with leading dimension ld; its order is ns[b] <= nmax.
// ---------------------------------------------------------------------------
template <typename T>
struct MatBatch {
    T* p;
    int ld;
    long long stride;
    __device__ __host__ T* at(int b) const { return p + (long long)b * stride; }
};

template <typename T>
struct VecBatch {
    T* p;
    long long stride;
    __device__ __host__ T* at(int b) const { return p + (long long)b * stride; }
};
