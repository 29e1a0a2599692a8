/*
 * fdk.h - C ABI of the MI355X (gfx950) FDK cone-beam back-projection library.
 *
 * The method is the back-projection stage of FDK as restated by Chen et al.,
 * "iFDK: A Scalable Framework for Instant High-resolution Image
 * Reconstruction" (SC'19): every voxel is mapped through each view's
 * projection geometry (Eq. 1, Eq. 2), the filtered projection is sampled
 * bilinearly (Alg. 3) and the distance-weighted sample is accumulated into
 * the volume (Alg. 2), using the reduced-cost coordinate scheme of Alg. 4
 * (Theorems 1-3: u and z are constant along a z-column, v is linear in k,
 * mirrored slices share v).
 *
 * Conventions shared by every entry point
 *  - Lengths share one unit (Table 1 mixes "pixel" and "mm"; Eq. 3 adds d to
 *    D_x * index, so they must agree).
 *  - Volume arrays are (Nz_local, Ny, Nx) FP32, x fastest: element (i,j,k) of
 *    the slab is vol[((k_local * Ny) + j) * Nx + i].
 *  - Projection arrays are (nviews, Nv, Nu), u fastest: q[(s*Nv + v)*Nu + u]
 *    holds view view0+s.
 *  - Device pointers are HIP device (or managed) memory owned by the caller,
 *    who keeps them alive until the work on `stream` completes. Host
 *    pointers (the geometry and its angle array) are read during the call
 *    only and may be freed on return.
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *    Every call is asynchronous on that stream and allocates no device
 *    memory.
 *  - Errors: arguments are validated on the host before anything is
 *    enqueued. A failed call returns a non-zero fdk_status, enqueues nothing
 *    (except FDK_ERR_HIP, reported after a launch failed) and leaves a
 *    message for fdk_last_error() in the calling thread. No call aborts or
 *    throws across the ABI.
 */
#ifndef FDK_H_
#define FDK_H_

#include <stdint.h>

/* Exported entry points (the library hides every other symbol). */
#if defined(__GNUC__) || defined(__clang__)
#define FDK_API __attribute__((visibility("default")))
#else
#define FDK_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FDK_OK = 0,
  FDK_ERR_INVALID_ARG = 1, /* a pointer, size, range or geometry is invalid */
  FDK_ERR_UNSUPPORTED = 2, /* a dtype, filter or slab kind the library does not support */
  FDK_ERR_HIP = 3,         /* the HIP runtime reported an error */
  FDK_ERR_OUT_OF_MEMORY = 4
} fdk_status;

/* Storage type of filtered projections. Arithmetic is FP32 throughout. */
typedef enum { FDK_F32 = 0, FDK_F16 = 1, FDK_BF16 = 2 } fdk_dtype;

/* Ramp kernels of the filtering stage (Alg. 1; the paper defers F_ramp to
 * the FDK literature): Ram-Lak and Shepp-Logan, sampled at the detector
 * pitch scaled to the rotation axis. */
typedef enum { FDK_RAMLAK = 0, FDK_SHEPP_LOGAN = 1 } fdk_filter_kind;

/* Which global slices a volume buffer holds.
 * FDK_SLAB_CONTIGUOUS : slices [z0, z0 + nz_local) in order.
 * FDK_SLAB_MIRROR_PAIR: a mirrored pair of slabs as in the paper's 2R
 *   sub-volumes (Fig. 5): with h = nz_local / 2, slices [z0, z0 + h)
 *   followed by [Nz - z0 - h, Nz - z0), each in ascending global k. */
typedef enum { FDK_SLAB_CONTIGUOUS = 0, FDK_SLAB_MIRROR_PAIR = 1 } fdk_slab_kind;

/* flags: accumulate into the output instead of overwriting it. */
#define FDK_ACCUMULATE 1u
/* flags of fdk_backproject and fdk_forward_project: run the direct variant
 * (FP64 column coordinates, taps read from global memory) instead of the
 * LDS-tiled one. The library picks the direct variant by itself only when
 * a brick's detector footprint exceeds the LDS budget; the results agree up
 * to FP32 rounding. For comparisons and tests of that variant. */
#define FDK_DIRECT 4u
/* flags of fdk_sirt_iteration: clamp the updated volume at zero. */
#define FDK_NONNEG 2u
/* flags of fdk_forward_project: sum every finite brick in 32-bit fixed
 * point, also bricks with a wide range of magnitudes, which by default sum
 * in 64-bit fixed point or FP32 (see fdk_forward_project). Each pixel's
 * error is then at most half a unit of about 2^-31 K M per contribution
 * (K M bounds what one pixel can receive from the brick): relative to the
 * brick's largest contributions rather than each pixel's own. Wide-range
 * volumes run up to twice as fast. The iterative entry points
 * (fdk_sirt_iteration, fdk_mlem_iteration) project this way. */
#define FDK_FIXED_SUMS 8u

/* Circular-orbit cone-beam geometry (Table 1; projection matrix Eq. 2).
 * The volume centre (voxel ((Nx-1)/2, (Ny-1)/2, (Nz-1)/2)) is on the
 * rotation axis; the principal point is pixel ((Nu-1)/2 + off_u,
 * (Nv-1)/2 + off_v); view s is taken at gantry angle angles[s]. */
typedef struct {
  int32_t nx, ny, nz;    /* full volume, voxels */
  double dx, dy, dz;     /* voxel pitch */
  int32_t nu, nv;        /* detector, pixels */
  double du, dv;         /* pixel pitch */
  double off_u, off_v;   /* principal-point shift, pixels (0 in the paper) */
  double sod;            /* d: source to rotation axis */
  double sdd;            /* D: source to detector */
  int32_t np;            /* number of views in the scan */
  const double* angles;  /* HOST array of np gantry angles beta, radians */
} fdk_geometry;

/* Filtering stage, Alg. 1: for views [view0, view0 + nviews), multiply each
 * line-integral image by the cosine weight D / sqrt(D^2 + a^2 + b^2) (a, b:
 * the pixel's offset from the principal point on the detector) and convolve
 * every detector row (linear convolution, zero outside the row) with the
 * ramp kernel h sampled at tau = Du * d / D:
 *     Q(u) = tau * sum_n h(u - n) * E~(n).
 * e: device FP32 (nviews, Nv, Nu). q: device (nviews, Nv, Nu) of out_dtype,
 * must not overlap e. The FDK constant pi * d^2 / Np is NOT applied here (it
 * is fdk_backproject's `scale`), which keeps 16-bit storage in range.
 * Errors: FDK_ERR_INVALID_ARG for a bad geometry, range or null pointer;
 * FDK_ERR_UNSUPPORTED for an unknown kind or dtype, or Nu above 8192. */
FDK_API fdk_status fdk_filter(const fdk_geometry* g, int32_t view0, int32_t nviews,
                      const float* e, void* q, fdk_dtype out_dtype,
                      fdk_filter_kind kind, void* stream);

/* The filtering stage of fdk_filter on a band of detector rows: rows
 * [v0, v0 + nrows) of views [view0, view0 + nviews). Element (s, r, u) of
 * the band is e[s * e_view_stride + r * Nu + u] on input and
 * q[s * q_view_stride + r * Nu + u] on output (strides in elements), so the
 * output may be the band's rows inside a full (nviews, Nv, Nu) array. Each
 * row's result equals fdk_filter's for the same detector row. Used to filter
 * only the rows a volume slab projects to.
 * Errors: as fdk_filter, plus FDK_ERR_INVALID_ARG for a band outside
 * [0, Nv) or a view stride smaller than nrows * Nu. */
FDK_API fdk_status fdk_filter_rows(const fdk_geometry* g, int32_t view0, int32_t nviews, int32_t v0,
                           int32_t nrows, const float* e, int64_t e_view_stride, void* q,
                           int64_t q_view_stride, fdk_dtype out_dtype, fdk_filter_kind kind,
                           void* stream);

/* Adjoint (transpose) of fdk_filter for FP32 gradients: for all E and G,
 *     <fdk_filter(E), G> = <E, fdk_filter_adjoint(G)>.
 * The ramp kernel is even, so the row convolution is its own transpose; the
 * cosine weight, applied before the convolution in fdk_filter, multiplies
 * the convolution's output here:
 *     E_grad(u) = F_cos(u, v) * tau * sum_n h(u - n) * G(n).
 * q_grad, e_grad: device FP32 (nviews, Nv, Nu), not overlapping. Used to
 * differentiate a reconstruction with respect to the line integrals.
 * Errors: as fdk_filter. */
FDK_API fdk_status fdk_filter_adjoint(const fdk_geometry* g, int32_t view0, int32_t nviews,
                                      const float* q_grad, float* e_grad, fdk_filter_kind kind,
                                      void* stream);

/* Back-projection, Alg. 2 computed as Alg. 4. For every voxel (i, j, k)
 * the slab holds, with [x, y, z] = P_s [i, j, k, 1], f = 1/z, W = f^2,
 * (u, v) = (x f, y f):
 *     vol(i,j,k) (+)= scale * sum_{s in [view0, view0+nviews)} W * interp2(Q_s, u, v)
 * interp2 is Alg. 3 with floor for int() and taps outside the detector
 * reading zero. q: device (nviews, Nv, Nu) of q_dtype (FP32, FP16 or BF16;
 * accumulation is FP32). vol: device FP32 slab, see fdk_slab_kind; z0 and
 * nz_local select its global slices. Without FDK_ACCUMULATE the slab is
 * overwritten (nviews = 0 then zeroes it). For FDK pass
 * scale = fdk_fdk_scale(g). Each voxel is owned by one thread that sums the
 * views in a fixed order: results are bitwise reproducible run to run.
 * Errors: FDK_ERR_INVALID_ARG for a null pointer, non-positive size, view
 * range outside [0, np), slab outside the volume (or an odd nz_local /
 * overlapping halves for a mirror pair), sod not larger than the volume's
 * half-diagonal in x-y (some z <= 0, Eq. 3), sdd not larger than sod (the
 * detector must lie beyond the rotation axis, Table 1), or a non-finite value. */
FDK_API fdk_status fdk_backproject(const fdk_geometry* g, int32_t view0, int32_t nviews,
                           const void* q, fdk_dtype q_dtype, float* vol,
                           int32_t z0, int32_t nz_local, fdk_slab_kind slab,
                           float scale, uint32_t flags, void* stream);

/* Forward projection: the exact adjoint (transpose) of fdk_backproject with
 * the same geometry, views, slab and scale, i.e. for all q and x
 *     <fdk_backproject(q), x> = <q, fdk_forward_project(x)>.
 * Every voxel of the slab adds scale * W * w_tap * vol(i,j,k) to each of its
 * four bilinear taps that lies inside the detector, with the identical
 * coordinates and weights the back-projector uses. vol: device FP32 slab.
 * q: device FP32 (nviews, Nv, Nu), overwritten unless FDK_ACCUMULATE.
 * Within a workgroup the splats are summed in 32-bit fixed point, scaled per
 * brick and view so that no partial sum can overflow. A brick with a wide
 * range of magnitudes (more than 1 % of its non-zero voxels below 2^-13 of
 * its largest) sums in 64-bit fixed point instead (half a unit of about
 * 2^-63 K M per contribution: a voxel 2^-40 of the largest reaches a pixel
 * through a full-weight tap at about FP32 precision of its own size), and a
 * brick holding NaN or infinity, or spanning more than 2^40, sums in FP32
 * (unless FDK_FIXED_SUMS, which keeps every finite brick in 32 bits). The workgroups' sums
 * meet in FP32 atomics, so the last bits vary from run to run.
 * Errors: as fdk_backproject. */
FDK_API fdk_status fdk_forward_project(const fdk_geometry* g, int32_t view0, int32_t nviews,
                               const float* vol, int32_t z0, int32_t nz_local,
                               fdk_slab_kind slab, float* q, float scale,
                               uint32_t flags, void* stream);

/* Detector rows that fdk_backproject reads for a slab (same z0, nz_local,
 * slab as there), over all np views of the scan: the rows of the bilinear
 * taps of every voxel of the slab (Alg. 3), plus one spare row on each side.
 * Rows outside these bands never reach the slab, so a reconstruction that
 * streams projections may filter (fdk_filter_rows) and keep only these.
 * On success band = {v0_a, n_a, v0_b, n_b}: rows [v0_a, v0_a + n_a) and
 * [v0_b, v0_b + n_b), ascending and disjoint, with n_b = 0 when one band
 * covers the slab (a contiguous slab, or mirror halves whose bands touch)
 * and n_a = 0 too when the slab projects off the detector. Host-only: no
 * device work. band is a host array of 4 int32.
 * Errors: as fdk_backproject for the geometry and slab; FDK_ERR_INVALID_ARG
 * for a null band. */
FDK_API fdk_status fdk_slab_rows(const fdk_geometry* g, int32_t z0, int32_t nz_local,
                         fdk_slab_kind slab, int32_t band[4]);

/* Iterative reconstruction with the matched pair (the paper names iterative
 * methods, which call the back-projection repeatedly, as a use of it): SIRT
 * (simultaneous iterative reconstruction, Gilbert 1972) with F =
 * fdk_forward_project and B = fdk_backproject at scale 1 over views
 * [view0, view0 + nviews) and the slab (z0, nz_local, slab as in
 * fdk_backproject):
 *     x <- x + lambda * C * B(R * (p - F x)),
 * R = 1 / max(F 1, 1e-3 max(F 1)) per detector pixel and
 * C = 1 / max(B 1, 1e-3 max(B 1)) per voxel (the inverse row and column
 * sums of F; raising sums below 1e-3 of the largest keeps the weights
 * continuous where rays or voxels are barely covered).
 *
 * fdk_sirt_weights writes R into row_inv (device FP32 (nviews, Nv, Nu)) and
 * C into col_inv (device FP32 slab); vol_tmp is a slab-sized device
 * workspace whose contents are overwritten. */
FDK_API fdk_status fdk_sirt_weights(const fdk_geometry* g, int32_t view0, int32_t nviews,
                                    int32_t z0, int32_t nz_local, fdk_slab_kind slab,
                                    float* row_inv, float* col_inv, float* vol_tmp, void* stream);

/* One SIRT iteration on x (device FP32 slab, updated in place) for measured
 * projections p (device FP32 (nviews, Nv, Nu)) and weights from
 * fdk_sirt_weights. flags: 0 or FDK_NONNEG. proj_tmp (projection-sized) and
 * vol_tmp (slab-sized) are device workspaces; neither may alias an input.
 * Errors: as fdk_backproject, plus FDK_ERR_INVALID_ARG for a null or
 * aliased buffer, a non-finite lambda or unknown flags. */
FDK_API fdk_status fdk_sirt_iteration(const fdk_geometry* g, int32_t view0, int32_t nviews,
                                      const float* p, const float* row_inv, const float* col_inv,
                                      float* x, int32_t z0, int32_t nz_local, fdk_slab_kind slab,
                                      float lambda, uint32_t flags, float* proj_tmp,
                                      float* vol_tmp, void* stream);

/* fdk_sirt_iteration without workspace arguments, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation): proj_tmp and vol_tmp come from a
 * static per-GPU array of 2^24 floats (64 MiB) that the library holds from
 * its load until the process ends, so the call allocates nothing. The
 * projections of the view range, rounded up to 64 floats, plus the slab's
 * voxels must fit that array, else FDK_ERR_INVALID_ARG. Every call on one
 * GPU shares its array: calls that overlap on a GPU (on different streams
 * or threads) race and must be ordered by the caller. Other arguments and
 * errors: as fdk_sirt_iteration, plus FDK_ERR_HIP if the array's device
 * address cannot be obtained. */
FDK_API fdk_status fdk_sirt_iteration_noalloc(const fdk_geometry* g, int32_t view0,
                                              int32_t nviews, const float* p,
                                              const float* row_inv, const float* col_inv,
                                              float* x, int32_t z0, int32_t nz_local,
                                              fdk_slab_kind slab, float lambda, uint32_t flags,
                                              void* stream);

/* One MLEM iteration (maximum-likelihood expectation maximisation, Shepp
 * and Vardi 1982; another of the iterative methods the paper names as users
 * of the back-projection) on x (device FP32 slab, updated in place) for
 * measured projections p (device FP32 (nviews, Nv, Nu)), with the same
 * matched pair, views and slab as fdk_sirt_iteration:
 *     x <- x * C * B(p / max(F x, 1e-3 max(F x))),
 * and a ratio of 0 where that denominator is 0. C is col_inv from
 * fdk_sirt_weights (the inverse column sums 1 / B 1, raised as there).
 * MLEM's domain is non-negative: x and p must hold no negative values (not
 * checked); a positive start (e.g. all ones) stays positive where the
 * volume is seen. proj_tmp (projection-sized) and vol_tmp (slab-sized) are
 * device workspaces whose contents are overwritten; neither may alias an
 * input. Errors: as fdk_sirt_iteration. */
FDK_API fdk_status fdk_mlem_iteration(const fdk_geometry* g, int32_t view0, int32_t nviews,
                                      const float* p, const float* col_inv, float* x, int32_t z0,
                                      int32_t nz_local, fdk_slab_kind slab, float* proj_tmp,
                                      float* vol_tmp, void* stream);

/* The 3 x 4 projection matrix P_s of Eq. 2 that every kernel uses for view
 * `view` (angle g->angles[view]), in the reduced form of Eq. 3 and
 * Theorems 2-3: for voxel (i, j, k), [x, y, z] = P [i, j, k, 1] with z the
 * depth along the central ray (the geometry's length unit) and
 * (u, v) = (x / z, y / z) in detector pixels. P: host array of 12 doubles,
 * row-major, owned by the caller. Host-only: validates g and view like the
 * other calls and makes no HIP call. Errors: FDK_ERR_INVALID_ARG for an
 * invalid geometry, a view outside [0, np) or a null P. */
FDK_API fdk_status fdk_projection_matrix(const fdk_geometry* g, int32_t view, double* P);

/* pi * d^2 / Np: the FDK constant (1/2) * (2 pi / Np) * d^2 of a full
 * 360-degree scan, since W = 1/z^2 carries no d^2. Returns NaN for a null
 * or invalid geometry. */
FDK_API double fdk_fdk_scale(const fdk_geometry* g);

/* Message describing the calling thread's most recent failed call ("" if
 * none). Valid until that thread's next call into the library. */
FDK_API const char* fdk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDK_H_ */
