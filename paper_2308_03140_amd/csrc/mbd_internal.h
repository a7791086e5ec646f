// Internal definitions shared by the HIP kernels and the host runtime of
// libmbd_hip.so.  Not part of the public C ABI (see include/mbd.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#define MBD_TILE 64          // SYMV / assembly tile edge (rows of one wavefront)
#define MBD_THREADS 256      // 4 wavefronts of 64 lanes
#define MBD_MAX_BATCH 65535  // matrices of one batched launch sequence (grid z)

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
#define MBD_ST_NOT_CONVERGED 8u    // the FP64 refinement missed its target

static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
static inline long long ceil_div_ll(long long a, long long b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Cross-lane primitives on the VALU (no LDS round trip).  DPP row
// permutations act within 16-lane rows: quad xor 1, quad xor 2, the mirror of
// each 8-lane half (lane l <-> 7 - l) and of each row (l <-> 15 - l).  The
// permlane swaps exchange rows between two registers: swap32(a, b) leaves
// a = [a lanes 0-31, b lanes 0-31], b = [a lanes 32-63, b lanes 32-63];
// swap16(a, b) leaves a = [a row 0, b row 0, a row 2, b row 2] and
// b = [a row 1, b row 1, a row 3, b row 3].
// ---------------------------------------------------------------------------
#define DPP_QUAD_XOR1 0xB1
#define DPP_QUAD_XOR2 0x4E
#define DPP_HALF_MIRROR 0x141
#define DPP_ROW_MIRROR 0x140
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned x) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __builtin_bit_cast(float, dpp_u32<CTRL>(__builtin_bit_cast(unsigned, x)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = dpp_u32<CTRL>((unsigned)u), hi = dpp_u32<CTRL>((unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// (the swap results are copied to scalars before the bit cast: a bit cast
// applied directly to an element of the returned vector reads element 0)
__device__ __forceinline__ void swap32(float& a, float& b) {
    auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b), false,
                                              false);
    const unsigned r0 = r[0], r1 = r[1];
    a = __builtin_bit_cast(float, r0);
    b = __builtin_bit_cast(float, r1);
}
__device__ __forceinline__ void swap16(float& a, float& b) {
    auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b), false,
                                              false);
    const unsigned r0 = r[0], r1 = r[1];
    a = __builtin_bit_cast(float, r0);
    b = __builtin_bit_cast(float, r1);
}
__device__ __forceinline__ void swap32(double& a, double& b) {
    const unsigned long long ua = __builtin_bit_cast(unsigned long long, a), ub = __builtin_bit_cast(unsigned long long, b);
    auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    const unsigned long long na = ((unsigned long long)(unsigned)hi[0] << 32) | (unsigned)lo[0];
    const unsigned long long nb = ((unsigned long long)(unsigned)hi[1] << 32) | (unsigned)lo[1];
    a = __builtin_bit_cast(double, na);
    b = __builtin_bit_cast(double, nb);
}
__device__ __forceinline__ void swap16(double& a, double& b) {
    const unsigned long long ua = __builtin_bit_cast(unsigned long long, a), ub = __builtin_bit_cast(unsigned long long, b);
    auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
    auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    const unsigned long long na = ((unsigned long long)(unsigned)hi[0] << 32) | (unsigned)lo[0];
    const unsigned long long nb = ((unsigned long long)(unsigned)hi[1] << 32) | (unsigned)lo[1];
    a = __builtin_bit_cast(double, na);
    b = __builtin_bit_cast(double, nb);
}

// Pairwise reduction steps of a multi-value butterfly.  Each takes two values
// x, y per lane and returns, in lanes where the named lane bit is 0, x summed
// over the lane pair that differs in that bit (with the bits below it for the
// mirror forms), and y in lanes where it is 1.
template <typename T>
__device__ __forceinline__ T pair_sum_b5(T x, T y) { swap32(x, y); return x + y; }
template <typename T>
__device__ __forceinline__ T pair_sum_b4(T x, T y) { swap16(x, y); return x + y; }
template <typename T>
__device__ __forceinline__ T pair_sum_b3(T x, T y) {
    const bool hi = (threadIdx.x & 8) != 0;
    return (hi ? y : x) + dpp<DPP_ROW_MIRROR>(hi ? x : y);
}
template <typename T>
__device__ __forceinline__ T pair_sum_b2(T x, T y) {
    const bool hi = (threadIdx.x & 4) != 0;
    return (hi ? y : x) + dpp<DPP_HALF_MIRROR>(hi ? x : y);
}
// full sum over lane bits 1 and 0
template <typename T>
__device__ __forceinline__ T quad_sum(T v) {
    v += dpp<DPP_QUAD_XOR2>(v);
    return v + dpp<DPP_QUAD_XOR1>(v);
}

// ---------------------------------------------------------------------------
// Wavefront / block reductions (deterministic: a fixed butterfly whose two
// operands every lane of a pair adds in the same order, so every lane sees
// bit-identical values)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v = quad_sum(v);
    v += dpp<DPP_HALF_MIRROR>(v);
    v += dpp<DPP_ROW_MIRROR>(v);
    T a = v, b = v;
    swap16(a, b);
    v = a + b;
    a = v; b = v;
    swap32(a, b);
    return a + b;
}

// Product over the wavefront, with the same butterfly (bit-identical in
// every lane).
__device__ __forceinline__ double wave_prod(double v) {
    v *= dpp<DPP_QUAD_XOR1>(v);
    v *= dpp<DPP_QUAD_XOR2>(v);
    v *= dpp<DPP_HALF_MIRROR>(v);
    v *= dpp<DPP_ROW_MIRROR>(v);
    double a = v, b = v;
    swap16(a, b);
    v = a * b;
    a = v; b = v;
    swap32(a, b);
    return a * b;
}

// Sixteen sums at once: returns in lane l the sum over the wave of v[l >> 2].
template <typename T>
__device__ __forceinline__ T wave_sum16(const T (&v)[16]) {
    T u[8], w[4];
#pragma unroll
    for (int i = 0; i < 8; i++) u[i] = pair_sum_b5(v[i], v[i + 8]);
#pragma unroll
    for (int i = 0; i < 4; i++) w[i] = pair_sum_b4(u[i], u[i + 4]);
    const T z0 = pair_sum_b3(w[0], w[2]), z1 = pair_sum_b3(w[1], w[3]);
    return quad_sum(pair_sum_b2(z0, z1));
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
// value of v in lane l (l wave-uniform) in every lane
__device__ __forceinline__ float lane_value(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

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
