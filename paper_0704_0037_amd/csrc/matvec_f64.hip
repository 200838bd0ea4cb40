// Interaction-matrix product, double precision: kernel instantiations and launch, and the product
// entry point that allocates nothing (its intermediates live in a fixed device array).
#include <mutex>
#include <string>

#include "matvec_launch.hpp"

namespace dda {

bool beam_ok(const dda_beam *b);

dda_status matvec_materials(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, double2 *dots,
                            hipStream_t s, const int *done, hipEvent_t *ev);

template <>
dda_status matvec_device<double>(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, double2 *dots,
                              hipStream_t s, const int *done, hipEvent_t *ev) {
    if (wrapped(c)) return matvec_materials(c, x, y, nrhs, scale, dots, s, done, ev);
    return matvec_device_impl<double>(c, x, y, nrhs, scale, dots, s, done, ev);
}

// the unit-polarizability product of an inhomogeneous particle (the materials enter around it)
dda_status matvec_device_unit(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, hipStream_t s,
                              const int *done, hipEvent_t *ev) {
    return matvec_device_impl<double>(c, x, y, nrhs, scale, nullptr, s, done, ev);
}

// ------------------------------------------------------------------ product without allocation
// Work memory of dda_matvec_noalloc: the x-pass and y-pass intermediates and the scale of one
// right-hand side, carved from this fixed array (each device holds its own copy for the life of
// the process).  Host code never passes the array's name to a kernel: it uses the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// device address of `scratch` on the current device, resolved once per device
dda_status scratch_address(void **out) {
    int dev = 0;
    DDA_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("dda_matvec_noalloc: device index out of range");
        return DDA_EINVAL;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        DDA_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return DDA_OK;
}

__global__ void k_put_scale(double2 *p, double re, double im) { *p = make_double2(re, im); }
}  // namespace

// bytes of scratch the product of one vector on this context needs: B1, B2, scale (256-aligned)
size_t noalloc_bytes(const Ctx &c) {
    const size_t b1 = (size_t)3 * c.nz * c.Lx * row_pitch(c.ny) * sizeof(double2);
    const size_t b2 = (size_t)3 * row_pitch(c.nz) * c.Lx * c.Ly * sizeof(double2);
    return round256(b1) + round256(b2) + round256(sizeof(double2));
}

}  // namespace dda

using namespace dda;

extern "C" dda_status dda_matvec_noalloc(dda_ctx *h, const dda_beam *beam, const void *x, void *y) {
    clear_error();
    Ctx *c = cx(h);
    if (!c || !beam || !x || !y) {
        set_error("dda_matvec_noalloc: NULL argument");
        return DDA_EINVAL;
    }
    if (x == y) {
        set_error("dda_matvec_noalloc: x and y must not overlap");
        return DDA_EINVAL;
    }
    if (!beam_ok(beam)) {
        set_error("dda_matvec_noalloc: beam without unit vectors");
        return DDA_EINVAL;
    }
    if (wrapped(*c)) {
        set_error("dda_matvec_noalloc: homogeneous contexts only (several materials or CLDR keep scaled vectors in "
                  "the context)");
        return DDA_ENOTSUP;
    }
    const size_t need = noalloc_bytes(*c);
    if (need > kScratchBytes) {
        set_error("dda_matvec_noalloc: the product of this particle needs " + std::to_string(need >> 20) +
                  " MiB of work memory, above the fixed " + std::to_string(kScratchBytes >> 20) + " MiB");
        return DDA_EINVAL;
    }
    void *base = nullptr;
    dda_status st = scratch_address(&base);
    if (st != DDA_OK) return st;
    unsigned char *p = static_cast<unsigned char *>(base);
    Work<double> wk;
    wk.nrhs = 1;
    wk.B1 = reinterpret_cast<double2 *>(p);
    p += round256((size_t)3 * c->nz * c->Lx * row_pitch(c->ny) * sizeof(double2));
    wk.B2 = reinterpret_cast<double2 *>(p);
    p += round256((size_t)3 * row_pitch(c->nz) * c->Lx * c->Ly * sizeof(double2));
    wk.scale = reinterpret_cast<double2 *>(p);
    double ar, ai;
    polarizability(*c, *beam, ar, ai);
    const double inv = 1.0 / ((double)c->Lx * c->Ly * c->Lz);
    hipLaunchKernelGGL(k_put_scale, dim3(1), dim3(1), 0, c->stream, wk.scale, ar * inv, ai * inv);
    return matvec_device_impl<double>(*c, (const double2 *)x, (double2 *)y, 1, wk.scale, nullptr, c->stream, nullptr,
                                      nullptr, &wk);
}
