// Internal state of one DDA context (one particle on one GPU) and the launch helpers shared by
// the matvec, solver and read-out translation units.
#pragma once

#include <type_traits>

#include <numeric>
#include <vector>

#include "dda.h"
#include "fft.hpp"

namespace dda {

// every exported call starts with it, so the thread's error message describes that call only
void clear_error();

// Work buffers of one precision, sized for `nrhs` right-hand sides.
template <typename R> struct Work {
    int nrhs = 0;
    cplx<R> *B1 = nullptr;   // [3 nrhs][nz][Lx][row_pitch(ny)]
    cplx<R> *B2 = nullptr;   // [Lx][3 nrhs][Ly][row_pitch(nz)]
    cplx<R> *scale = nullptr;  // [nrhs] alpha / (Lx Ly Lz)
    cplx<R> *dots = nullptr;   // per-block partial sums of the matvec epilogue
    size_t ndots = 0;
};

// lines per block of the x and y passes (powers of two) and their log2
struct Tiles {
    int nl_x = 0, nl_y = 0, lnl_x = 0, lnl_y = 0;
};

struct Ctx {
    int nx = 0, ny = 0, nz = 0;
    int Lx = 0, Ly = 0, Lz = 0;
    int64_t N = 0;
    double m_re = 0, m_im = 0, kd = 0;
    int polarizability = DDA_POL_LDR;
    hipStream_t stream = nullptr;      // the caller's stream (all calls are ordered on it)
    hipStream_t own_stream = nullptr;  // the context's own stream: solves run (and graphs capture) here
    Tiles tl64, tl32;                  // lines per block of the x / y passes, per precision
    int nc_z = 0;                      // columns per block (z pass)

    std::vector<uint8_t> mask;      // host copy [nz][ny][nx]
    std::vector<int32_t> lin_host;  // linear cell index of each dipole

    int *gmap = nullptr;            // device [nz][ny][nx] -> dipole index or -1
    int2 *rows = nullptr;           // device [nz][ny] single-run descriptors of the rows (x passes)
    // a batch of particles on one grid (pack_setup): gmap and rows hold one map per right-hand side,
    // these many elements apart (0 for a single particle); the tensor, twiddles and plans are
    // borrowed from the member whose grid is the batch's
    size_t gmap_stride = 0, rows_stride = 0;
    bool borrowed = false;
    int *lin = nullptr;             // device [N] linear cell index
    int *line_start = nullptr;      // device [ny*nz + 1] first dipole of each (y, z) line (read-out)
    double2 *ghat = nullptr;        // device octant tensor, fp64
    float2 *ghat32 = nullptr;       // device octant tensor, fp32 (optional)
    double2 *tw64 = nullptr;        // twiddle tables, fp64
    float2 *tw32 = nullptr;         // twiddle tables, fp32
    FftPlan pxf{}, pxi{}, pyf{}, pyi{}, pzf{}, pzi{};

    Work<double> w64;
    Work<float> w32;

    // solver scratch
    double2 *vecs = nullptr;    // Krylov vectors, fp64
    size_t vecs_elems = 0;
    float2 *vecs32 = nullptr;
    size_t vecs32_elems = 0;
    double *sbuf = nullptr;     // device scalar state + reduction partials
    size_t sbuf_bytes = 0;
    double *hbuf = nullptr;     // pinned host mirror for convergence checks
    size_t hbuf_bytes = 0;
    double2 *red = nullptr;     // read-out partials
    size_t red_elems = 0;
    void *snap = nullptr;       // state of a relaxed-precision solve at its switch (rolled back on stall)
    size_t snap_bytes = 0;

    // a double-precision solve that stopped at its iteration limit leaves its complete state in
    // vecs / sbuf and can be continued (dda_solve with opts.resume): its batch size and method
    // (resume_nrhs = 0: nothing to continue)
    int resume_nrhs = 0;
    int resume_solver = -1;
    uint64_t resume_beams = 0;  // hash of the beams of that solve (a continuation needs the same ones)

    // inhomogeneous particle (dda_setup_materials, nmat > 1) or CLDR (a diagonal polarizability
    // tensor): mask values name the material of each cell; the product runs with unit
    // polarizability between a scaling by beta of each dipole's material and component and back
    // (the solver's per-RHS scales and beta are then 1)
    int nmat = 1;
    std::vector<double> mat_re, mat_im;  // refractive index of each material
    uint8_t *dmat = nullptr;             // device [N] material of each dipole (0-based)
    double2 *mat_beta = nullptr;         // device [rows][nmat][3] beta per right-hand side, material, component
    int mat_beta_rows = 0;
    double2 *xtmp = nullptr;             // device [rows][3][N] scaled vectors
    int xtmp_rows = 0;
};

// whether the product runs wrapped between per-dipole scalings (several materials, or CLDR)
inline bool wrapped(const Ctx &c) { return c.nmat > 1 || c.polarizability == DDA_POL_CLDR; }
// set up the wrapping for a context made by setup(): n_mat refractive indices m [n_mat][2]
dda_status material_init(Ctx &c, int n_mat, const double *m);

// inhomogeneous particles: beta of every material for the beams (device table, rows = n), and the
// scaled-vector buffer for at least max(n, 2) vectors; call before a solve's graphs are captured
dda_status material_prepare(Ctx &c, const dda_beam *beams, int n);
// P = beta x for one vector [3][N] of a beam (P may be c.xtmp rows)
dda_status material_scale(Ctx &c, const dda_beam &b, const double2 *x, double2 *P, hipStream_t s);
// Cabs of the dipole polarizations P [3][N] of a beam: per material (-Im(1/alpha) - 2k^3/3) |P|^2
dda_status material_cabs(Ctx &c, const dda_beam &b, const double2 *P, double &cabs);
// alpha of material m (refractive index m_re + i m_im) for a beam
void polarizability_of(const Ctx &c, const dda_beam &b, double m_re, double m_im, double &re, double &im);
// component comp (0..2) of the diagonal polarizability (CLDR; the scalar alpha otherwise)
void polarizability_comp(const Ctx &c, const dda_beam &b, double m_re, double m_im, int comp, double &re, double &im);

// the work buffers of precision R
template <typename R> inline Work<R> &work_of(Ctx &c) {
    if constexpr (std::is_same<R, double>::value) return c.w64;
    else return c.w32;
}

// alpha of the context's material for a beam (LDR depends on the beam); 1 for an inhomogeneous
// particle, whose polarizabilities enter through material_prepare / material_scale
void polarizability(const Ctx &c, const dda_beam &b, double &re, double &im);

// Matvec on nrhs vectors: y = A x; alphas [nrhs] host complex; optionally leaves per-block
// bilinear partial sums x.y in w.dots (one block range per right-hand side).
template <typename R>
dda_status matvec_launch(Ctx &c, const cplx<R> *x, cplx<R> *y, int nrhs, const double *alpha_re,
                         const double *alpha_im, bool want_dots, hipStream_t s);

template <typename R> dda_status ensure_work(Ctx &c, int nrhs);

// y = A x on device buffers with device scales [nrhs] (alpha / (Lx Ly Lz)); dots (nullable)
// receives per-block bilinear partial sums x.y; done (nullable) skips converged right-hand sides.
template <typename R>
dda_status matvec_device(Ctx &c, const cplx<R> *x, cplx<R> *y, int nrhs, const cplx<R> *scale, cplx<R> *dots,
                         hipStream_t s, const int *done, hipEvent_t *ev = nullptr);
template <>
dda_status matvec_device<double>(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, double2 *dots,
                                 hipStream_t s, const int *done, hipEvent_t *ev);
template <>
dda_status matvec_device<float>(Ctx &c, const float2 *x, float2 *y, int nrhs, const float2 *scale, float2 *dots,
                                hipStream_t s, const int *done, hipEvent_t *ev);
// double-precision x, y, scale and dots through single-precision transforms (context with fp32)
dda_status matvec_device_mixed(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, double2 *dots,
                               hipStream_t s, const int *done, hipEvent_t *ev = nullptr);

// number of per-block dot partials the x-inverse kernel writes per right-hand side
template <typename R> inline const Tiles &tiles_of(const Ctx &c) { return sizeof(R) == 8 ? c.tl64 : c.tl32; }
inline size_t max_dots_per_rhs(const Ctx &c) { return (size_t)3 * c.nz * c.ny; }
template <typename R> bool tiles_valid(const Ctx &c, int axis, int nl);
template <typename R> inline size_t dots_per_rhs(const Ctx &c) {
    const Tiles &t = tiles_of<R>(c);
    return (size_t)3 * c.nz * ((c.ny + t.nl_x - 1) / t.nl_x);
}

dda_status device_alloc(void **p, size_t bytes);

// the opaque ABI handle is the context itself
inline Ctx *cx(dda_ctx *p) { return reinterpret_cast<Ctx *>(p); }
inline const Ctx *cx(const dda_ctx *p) { return reinterpret_cast<const Ctx *>(p); }

}  // namespace dda
