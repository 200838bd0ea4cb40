// Host side of the interaction-matrix product: picks, for each axis, the kernels specialized for
// its padded length when one exists (index arithmetic folds to constants) or the general ones.
// Included by one translation unit per precision.
#pragma once

#include <mutex>
#include <set>
#include <tuple>

#include "ctx.hpp"
#include "matvec_kernels.hpp"


namespace dda {

template <typename R> inline const cplx<R> *tw_of(const Ctx &c);
template <> inline const double2 *tw_of<double>(const Ctx &c) { return c.tw64; }
template <> inline const float2 *tw_of<float>(const Ctx &c) { return c.tw32; }
template <typename R> inline const cplx<R> *ghat_of(const Ctx &c);
template <> inline const double2 *ghat_of<double>(const Ctx &c) { return c.ghat; }
template <> inline const float2 *ghat_of<float>(const Ctx &c) { return c.ghat32; }

// blocks above 64 KiB of dynamic LDS must be allowed explicitly; done once per kernel, device and
// size, so that launches recorded into a graph later make no attribute calls
template <class K> inline void allow_lds(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return;
    static std::mutex mu;
    static std::set<std::tuple<const void *, int, size_t>> seen;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const void *f = reinterpret_cast<const void *>(kernel);
    std::lock_guard<std::mutex> lock(mu);
    if (seen.insert(std::make_tuple(f, dev, bytes)).second)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

#define DDA_DISPATCH(LEN, KERNEL, BYTES, ...)                                          \
    switch (LEN) {                                                                     \
        DDA_SPECIALIZED_LENGTHS(DDA_CASE_##KERNEL)                                     \
        default:                                                                       \
            allow_lds(&KERNEL<R, 0>, BYTES);                                           \
            hipLaunchKernelGGL((KERNEL<R, 0>), __VA_ARGS__);                           \
            break;                                                                     \
    }
// the x passes also carry the precision of the vectors
#define DDA_DISPATCH_X(LEN, KERNEL, BYTES, ...)                                        \
    switch (LEN) {                                                                     \
        DDA_SPECIALIZED_LENGTHS(DDA_CASE_##KERNEL)                                     \
        default:                                                                       \
            allow_lds(&KERNEL<R, 0, RX>, BYTES);                                       \
            hipLaunchKernelGGL((KERNEL<R, 0, RX>), __VA_ARGS__);                       \
            break;                                                                     \
    }
#define DDA_CASE_k_fwd_x(L) case L: allow_lds(&k_fwd_x<R, L, RX>, DDA_BYTES); hipLaunchKernelGGL((k_fwd_x<R, L, RX>), DDA_ARGS); break;
#define DDA_CASE_k_fwd_y(L) case L: allow_lds(&k_fwd_y<R, L>, DDA_BYTES); hipLaunchKernelGGL((k_fwd_y<R, L>), DDA_ARGS); break;
#define DDA_CASE_k_zmul(L) case L: allow_lds(&k_zmul<R, L>, DDA_BYTES); hipLaunchKernelGGL((k_zmul<R, L>), DDA_ARGS); break;
#define DDA_CASE_k_inv_y(L) case L: allow_lds(&k_inv_y<R, L>, DDA_BYTES); hipLaunchKernelGGL((k_inv_y<R, L>), DDA_ARGS); break;
#define DDA_CASE_k_inv_x(L) case L: allow_lds(&k_inv_x<R, L, RX>, DDA_BYTES); hipLaunchKernelGGL((k_inv_x<R, L, RX>), DDA_ARGS); break;

// Transforms in precision R on the work buffers of precision R (the context's, or the
// intermediates B1 / B2 of `wk` when given); x, y, scale and dots in RX.
template <typename R, typename RX = R>
dda_status matvec_device_impl(Ctx &c, const cplx<RX> *x, cplx<RX> *y, int nrhs, const cplx<RX> *scale,
                              cplx<RX> *dots, hipStream_t s, const int *done, hipEvent_t *ev,
                              const Work<R> *wk = nullptr) {
    using C = cplx<R>;
    const Work<R> &w = wk ? *wk : work_of<R>(c);
    const C *tw = tw_of<R>(c);
    const C *gh = ghat_of<R>(c);
    const int ncomp = 3 * nrhs;
    const Tiles &tl = tiles_of<R>(c);
    const int nlx = tl.nl_x, nly = tl.nl_y;
    const int ytiles = (c.ny + nlx - 1) / nlx, ztiles = (c.nz + nly - 1) / nly;
    const size_t lx_bytes = (size_t)nlx * lds_line_stride(c.Lx) * sizeof(C);
    const size_t ly_bytes = (size_t)nly * lds_line_stride(c.Ly) * sizeof(C);
    const size_t lz_bytes = zmul_lds_elems(c.Lz) * sizeof(C);
    const int N = (int)c.N;
    if (ev) DDA_HIP_CHECK(hipEventRecord(ev[0], s));
#define DDA_ARGS dim3(ncomp * c.nz * ytiles), dim3(nlx * c.pxf.tpl), lx_bytes, s, c.gmap, c.rows, c.gmap_stride, \
                 c.rows_stride, x, w.B1, c.nx, c.ny, c.nz, N, \
                 c.pxf, tw, tl.lnl_x, done
#define DDA_BYTES lx_bytes
    DDA_DISPATCH_X(c.Lx, k_fwd_x, DDA_BYTES, DDA_ARGS)
#undef DDA_BYTES
#undef DDA_ARGS
    if (ev) DDA_HIP_CHECK(hipEventRecord(ev[1], s));
#define DDA_ARGS dim3(ncomp * c.Lx * ztiles), dim3(nly * c.pyf.tpl), ly_bytes, s, w.B1, w.B2, c.ny, c.nz, c.Lx, ncomp, \
                 c.pyf, tw, tl.lnl_y, done
#define DDA_BYTES ly_bytes
    DDA_DISPATCH(c.Ly, k_fwd_y, DDA_BYTES, DDA_ARGS)
#undef DDA_BYTES
#undef DDA_ARGS
    if (ev) DDA_HIP_CHECK(hipEventRecord(ev[2], s));
    const int zblocks = (c.Lx / 2 + 1) * (c.Ly / 2 + 1);  // one block per octant column
#define DDA_ARGS dim3((zblocks + 7) / 8 * 8), dim3(3 * zmul_ct(c.pzf)), lz_bytes, s, w.B2, gh, c.nz, \
                 c.Lx, c.Ly, nrhs, c.pzf, c.pzi, tw, done
#define DDA_BYTES lz_bytes
    DDA_DISPATCH(c.Lz, k_zmul, DDA_BYTES, DDA_ARGS)
#undef DDA_BYTES
#undef DDA_ARGS
    if (ev) DDA_HIP_CHECK(hipEventRecord(ev[3], s));
#define DDA_ARGS dim3(ncomp * c.Lx * ztiles), dim3(nly * c.pyi.tpl), ly_bytes, s, w.B2, w.B1, c.ny, c.nz, c.Lx, ncomp, \
                 c.pyi, tw, tl.lnl_y, done
#define DDA_BYTES ly_bytes
    DDA_DISPATCH(c.Ly, k_inv_y, DDA_BYTES, DDA_ARGS)
#undef DDA_BYTES
#undef DDA_ARGS
    if (ev) DDA_HIP_CHECK(hipEventRecord(ev[4], s));
#define DDA_ARGS dim3(ncomp * c.nz * ytiles), dim3(nlx * c.pxi.tpl), lx_bytes, s, c.gmap, c.rows, c.gmap_stride, \
                 c.rows_stride, w.B1, x, y, c.nx, c.ny, c.nz, \
                 N, c.pxi, tw, tl.lnl_x, scale, dots, done
#define DDA_BYTES lx_bytes
    DDA_DISPATCH_X(c.Lx, k_inv_x, DDA_BYTES, DDA_ARGS)
#undef DDA_BYTES
#undef DDA_ARGS
    if (ev) DDA_HIP_CHECK(hipEventRecord(ev[5], s));
    DDA_HIP_CHECK(hipGetLastError());
    return DDA_OK;
}

}  // namespace dda
