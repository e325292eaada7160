// Device-side helpers shared by the HIP kernels of libsv.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sv {

template <typename R> struct CT;
template <> struct CT<float> { using T = float2; };
template <> struct CT<double> { using T = double2; };
template <typename R> using cvec = typename CT<R>::T;

template <typename R>
__device__ __forceinline__ cvec<R> cmake(R re, R im) {
    cvec<R> z;
    z.x = re;
    z.y = im;
    return z;
}
template <typename R>
__device__ __forceinline__ cvec<R> cmul(cvec<R> a, cvec<R> b) {
    return cmake<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// u0 * a + u1 * b
template <typename R>
__device__ __forceinline__ cvec<R> cmac2(cvec<R> u0, cvec<R> a, cvec<R> u1, cvec<R> b) {
    return cmake<R>(u0.x * a.x - u0.y * a.y + u1.x * b.x - u1.y * b.y,
                    u0.x * a.y + u0.y * a.x + u1.x * b.y + u1.y * b.x);
}

// Up to 40 bit positions that are held fixed while enumerating the other
// bits of an index: expand() inserts a zero at each position (ascending)
// and then ORs in the fixed values.
struct Ins {
    int nf;
    uint8_t pos[40];
    uint64_t fval;
};

__device__ __forceinline__ uint64_t expand(uint64_t p, const Ins &f) {
    for (int i = 0; i < f.nf; ++i) {
        const int q = f.pos[i];
        const uint64_t lo = p & ((1ull << q) - 1ull);
        p = ((p >> q) << (q + 1)) | lo;
    }
    return p | f.fval;
}

// software bit deposit: scatter the low bits of x into the set bits of mask
__device__ __forceinline__ uint64_t pdep64(uint64_t x, uint64_t mask) {
    uint64_t r = 0;
    while (mask) {
        const uint64_t low = mask & (~mask + 1ull);
        if (x & 1ull) r |= low;
        x >>= 1;
        mask &= mask - 1ull;
    }
    return r;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// exp(2 pi i t / 2^64) for a phase held as an exact 64-bit fraction of a turn
__device__ __forceinline__ float2 turn_phase_f32(uint64_t t) {
    const float x = (float)(int64_t)t * 1.0842021724855044e-19f;   // 2^-63 half-turns
    float s, c;
    sincospif(x, &s, &c);
    return make_float2(c, s);
}
__device__ __forceinline__ double2 turn_phase_f64(uint64_t t) {
    const double x = (double)(int64_t)t * 1.0842021724855044e-19;  // 2^-63
    double s, c;
    sincospi(x, &s, &c);
    return make_double2(c, s);
}
template <typename R> __device__ __forceinline__ cvec<R> turn_phase(uint64_t t);
template <> __device__ __forceinline__ float2 turn_phase<float>(uint64_t t) { return turn_phase_f32(t); }
template <> __device__ __forceinline__ double2 turn_phase<double>(uint64_t t) { return turn_phase_f64(t); }

}  // namespace sv
