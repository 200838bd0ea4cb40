// Shared device/host helpers of the DDA library: complex arithmetic on HIP vector types,
// error plumbing.  Complex numbers are stored interleaved (re, im) as double2 / float2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <string>

namespace dda {

template <typename R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename R> using cplx = typename cvec<R>::type;

template <typename C> __host__ __device__ __forceinline__ C mk(decltype(C::x) re, decltype(C::x) im) {
    C c;
    c.x = re;
    c.y = im;
    return c;
}
template <typename C> __host__ __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __host__ __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __host__ __device__ __forceinline__ C cmul(C a, C b) {
    return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __host__ __device__ __forceinline__ C cmulc(C a, C b) {
    return mk<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __host__ __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return mk<C>(a.x * s, a.y * s); }
template <typename C> __host__ __device__ __forceinline__ C cconj(C a) { return mk<C>(a.x, -a.y); }
// multiply by -i (forward, DIR < 0) or +i (inverse, DIR > 0)
template <int DIR, typename C> __host__ __device__ __forceinline__ C mul_i(C a) {
    return DIR < 0 ? mk<C>(a.y, -a.x) : mk<C>(-a.y, a.x);
}
template <typename C> __host__ __device__ __forceinline__ C czero() { return mk<C>(0, 0); }

// Pitch (elements) of the rows of the product's intermediates along their contiguous axis (y in
// B1, z in B2): the cell count rounded up to 16, so that every row starts on a 256-byte boundary
// and the tiles of lines that the transposing passes store side by side fill whole 128-byte
// segments whatever the particle's size.
__host__ __device__ constexpr int row_pitch(int n) { return (n + 15) & ~15; }

// Streaming (non-temporal) global load and store of one complex value: the FFT passes read and
// write each intermediate element exactly once, so they bypass cache retention
template <typename C> __device__ __forceinline__ C ld_stream(const C *p) {
    typedef decltype(C::x) V2 __attribute__((ext_vector_type(2)));
    const V2 w = __builtin_nontemporal_load(reinterpret_cast<const V2 *>(p));
    return mk<C>(w.x, w.y);
}
template <typename C> __device__ __forceinline__ void st_stream(C *p, C v) {
    typedef decltype(C::x) V2 __attribute__((ext_vector_type(2)));
    V2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<V2 *>(p));
}
// complex value converted between precisions
template <typename D, typename S> __host__ __device__ __forceinline__ D ccast(S v) {
    return mk<D>((decltype(D::x))v.x, (decltype(D::x))v.y);
}

// Thread-local last error message, set by the ABI layer.
void set_error(const std::string &msg);

}  // namespace dda

#define DDA_HIP_CHECK(call)                                                              \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            char b_[512];                                                                \
            snprintf(b_, sizeof b_, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                     __FILE__, __LINE__);                                                \
            ::dda::set_error(b_);                                                        \
            return e_ == hipErrorOutOfMemory ? DDA_ENOMEM : DDA_EHIP;                     \
        }                                                                                \
    } while (0)
