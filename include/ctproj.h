/*
 * ctproj.h -- C ABI of the MI355X (gfx950) separable-footprint / distance-driven CT projector.
 *
 * The library computes the forward projection y = A x (paper, Section 2.3, Eq. 1) and the
 * matched back projection x = A^T y (Eq. 2) of a voxel volume for 2D fan-beam, 3D circular
 * cone-beam and 3D non-circular cone-beam scans (Section 2.2, Table 1), with flat or curved
 * (cylindrical, centred on the source) detectors.  Two projector models are provided
 * (Section 2.3): the separable footprint (SF; trapezoid x trapezoid, "SF-TT", in 3D) and
 * distance driven (DD).  The system matrix is never stored; every call recomputes it.
 *
 * Data layout (dense, caller-owned device memory, FP32):
 *   volume    [batch][nz][ny][nx]       x fastest   (2D: [batch][ny][nx])
 *   sinogram  [batch][n_views][nv][nu]  u fastest   (2D: [batch][n_views][nu])
 * Voxel (ix, iy, iz) is centred at (x_ofst + (ix-(nx-1)/2) dx, y_ofst + (iy-(ny-1)/2) dy,
 * z_ofst + (iz-(nz-1)/2) dz); detector column i at u = (i-(nu-1)/2) du - u_ofst and row j at
 * v = (j-(nv-1)/2) dv - v_ofst (Table 1).  At theta = 0 the source is at (x_src, SAD, z_src),
 * the detector centre at (0, SAD-SDD, 0), e_u = +x, e_v = +z; the gantry pose is
 * R = Rz(theta) Rx(phi) Ry(psi) (Section 2.2: rotation order y -> x -> z), all counter-
 * clockwise.  A curved detector is an arc of radius SDD about the source; u is arc length.
 *
 * Errors: every function returns a ctp_status; nothing throws across the ABI.  Argument and
 * geometry errors are detected before any device work and leave outputs untouched.
 * ctp_last_error() gives a thread-local description of the last failure.
 *
 * Threading: a plan is immutable after creation and may be used concurrently from several
 * host threads and streams, provided each concurrent call has its own workspace.
 */
#ifndef CTPROJ_H
#define CTPROJ_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CTP_OK = 0,
    CTP_EINVAL = -1,        /* bad argument, size or geometry (e.g. object at/behind source) */
    CTP_EUNSUPPORTED = -2,  /* valid request that this build does not implement */
    CTP_ENOMEM = -3,        /* device or host allocation failed */
    CTP_EDEVICE = -4,       /* HIP runtime / launch failure */
    CTP_ETIMEOUT = -5,      /* a wait ended before the work was done (ctserve.h) */
    CTP_ECANCELED = -6      /* the request was cancelled before it ran (ctserve.h) */
} ctp_status;

/* Scan kinds (Section 2.2). */
typedef enum { CTP_FAN2D = 0, CTP_CONE_CIRC = 1, CTP_CONE_NONCIRC = 2 } ctp_geom_kind;
/* Detector models (Section 1 and 2.3: curved detectors for 2D fan and 3D circular scans). */
typedef enum { CTP_DET_FLAT = 0, CTP_DET_CURVED = 1 } ctp_det;
/* Projector models (Section 2.3). */
typedef enum { CTP_SF = 0, CTP_DD = 1 } ctp_method;
/* Storage types of the caller's volume and sinogram buffers.  Arithmetic is FP32 in every
 * case: BF16 / FP16 inputs are widened on load, outputs are rounded to nearest even on store
 * (an FP16 value beyond 65504 becomes infinity). */
typedef enum { CTP_F32 = 0, CTP_BF16 = 1, CTP_F16 = 2 } ctp_dtype;
/* Direction of a call, for workspace queries. */
typedef enum { CTP_FORWARD = 0, CTP_BACKWARD = 1 } ctp_direction;
/* Projection modes (Section 2.3).  PROJ: the standard projector pair.  RECON: the back
 * projection of filtered back projection, with a depth-dependent weight per view: the SF
 * footprint of each voxel is used as an interpolation kernel normalised to unit sum and view
 * b is weighted by (SAD_b / W_b)^2, W_b the depth of the voxel centre (flat detector: distance
 * from the source along the detector normal; curved: in-plane distance from the source).  The
 * forward projection in RECON mode is the exact transpose of that back projection.  RECON is
 * built for SF on circular scans (2D fan, 3D circular cone; flat or curved). */
typedef enum { CTP_MODE_PROJ = 0, CTP_MODE_RECON = 1 } ctp_mode;
/* Ramp filter windows (ctp_ramp_filter). */
typedef enum { CTP_WINDOW_RAMLAK = 0, CTP_WINDOW_SHEPP_LOGAN = 1 } ctp_window;

/*
 * Geometry descriptor (Section 2.2, Table 1).  Each per-view parameter is a host pointer to
 * either one double (len == 1: every view shares it) or n_views doubles (len == n_views:
 * one value per view); a NULL pointer with len 0 means 0.0.  Angles in radians, lengths in
 * mm.  For CTP_FAN2D set nz = nv = 1 (dz, dv, z_src, z_ofst, v_ofst, phi, psi are ignored).
 * phi and psi must be zero unless kind == CTP_CONE_NONCIRC.  The descriptor is read only
 * during ctp_plan_create.
 */
typedef struct {
    ctp_geom_kind kind;
    ctp_det det;
    int32_t nx, ny, nz;
    double dx, dy, dz;
    int32_t nu, nv;
    double du, dv;
    int32_t n_views;
    const double *theta, *phi, *psi, *sad, *sdd, *x_src, *z_src,
                 *x_ofst, *y_ofst, *z_ofst, *u_ofst, *v_ofst;
    int32_t len_theta, len_phi, len_psi, len_sad, len_sdd, len_x_src, len_z_src,
            len_x_ofst, len_y_ofst, len_z_ofst, len_u_ofst, len_v_ofst;
} ctp_geometry_desc;

typedef struct ctp_plan ctp_plan;   /* opaque; immutable after creation */

/*
 * Expand the geometry per view in FP64 on the host (source, detector frame, projection
 * constants, DD driving axis), validate it, and upload the per-view table to the current
 * HIP device.  The plan is bound to that device.  The paper's Projector(geom, mode, method,
 * direction) maps to a plan of (geometry, method, mode) and the choice of ctp_project /
 * ctp_backproject.
 * Errors: CTP_EINVAL for an unknown method or mode, non-positive sizes or spacings, a len
 * field other than 0, 1 or n_views, a NULL pointer with a non-zero len, any corner of the
 * volume at or behind the source plane in some view, or (DD) a detector column ray parallel
 * to the driving planes; CTP_EUNSUPPORTED for a curved detector with a non-circular scan
 * (Section 2.3), a curved detector with a non-zero x_src, DD with a non-circular scan, RECON
 * mode other than SF on a circular scan, or a footprint wider than 16 detector columns;
 * CTP_ENOMEM / CTP_EDEVICE for allocation / upload failures.
 * On success *out owns a device table of 128 bytes per view.
 */
ctp_status ctp_plan_create(const ctp_geometry_desc *desc, ctp_method method, ctp_mode mode,
                           ctp_plan **out);

/* Free the plan's device table (the counterpart of the geometry object's lifetime, Section
 * 2.2; no computation).  The caller must ensure no call using it is in flight.  NULL is
 * accepted. */
ctp_status ctp_plan_destroy(ctp_plan *plan);

/* Bytes of `batch` volumes and of `batch` sinograms stored as dtype: the device memory a
 * caller (or the serving engine's admission) budgets for the data itself, which the library
 * never copies out of the caller's buffers (zero-copy tensor sharing, Section 3.2). */
ctp_status ctp_plan_bytes(const ctp_plan *plan, ctp_dtype dtype, int64_t batch,
                          size_t *vol_bytes, size_t *sino_bytes);

/* Device workspace (bytes) that ctp_project (dir = CTP_FORWARD) or ctp_backproject
 * (CTP_BACKWARD) needs for `batch` items with the given storage types: the per-call scratch of
 * evaluating Eq. 1 / Eq. 2 on the device, which the caller owns.  Forward: two floats
 * per item for its accumulator scale, one float per 8192-element block of each item for its
 * max |x|, one z-fastest FP32 copy of the volume, and an FP32 sinogram when the sinogram is
 * BF16/FP16 (each part rounded up to 256 bytes).
 * Backward: an FP32 copy of the sinogram scaled by the per-cell amplitude (not needed for 2D
 * SF with an FP32 sinogram), and an FP32 volume when the volume is BF16/FP16.  The contents
 * are scratch; nothing is kept between calls. */
ctp_status ctp_workspace_bytes(const ctp_plan *plan, ctp_direction dir, ctp_dtype vol_dtype,
                               ctp_dtype sino_dtype, int64_t batch, size_t *bytes);

/*
 * Forward projection (Eq. 1): sino = A vol, or sino += A vol when accumulate != 0.
 * vol, sino: device pointers in the layouts above, `batch` items (batch >= 1; the plan is
 * shared by all items, Section 1: batched, channelled tensors).  workspace: device pointer
 * of at least ctp_workspace_bytes(plan, CTP_FORWARD, vol_dtype, sino_dtype, batch) bytes,
 * owned by the caller and
 * not used by any other concurrent call; 256-byte alignment required.  Asynchronous on
 * `stream` (0 = null stream); returns after enqueueing.
 * The volume must be finite: the projector accumulates in 32-bit fixed point whose scale is
 * set per batch item from that item's max |vol| (relative resolution ~1e-9 of the largest
 * possible cell sum; items with max |vol| * footprint bound below ~2^-96 lose resolution).  An
 * item's result therefore does not depend on the other items of the batch.
 * Errors: CTP_EINVAL (NULL pointers, batch < 1 or too large -- 2D: more than 2^20 images,
 * 3D: batch x ceil(nv / 512) above 65535 -- unknown dtype, workspace too small or misaligned,
 * plan used on another device), CTP_EDEVICE (launch).
 */
ctp_status ctp_project(const ctp_plan *plan, const void *vol, ctp_dtype vol_dtype,
                       void *sino, ctp_dtype sino_dtype, int64_t batch, int accumulate,
                       void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * ctp_project without a workspace argument and without any device allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the workspace is a static array of the library,
 * 96 MiB (100663296 bytes) per device, which each device that loads the library holds until
 * the process ends.  Same arguments, layouts, results and errors as ctp_project, plus
 * CTP_EINVAL when the call's forward workspace (ctp_workspace_bytes) exceeds 96 MiB (e.g. one
 * 256^3 FP32 volume fits, two do not) and CTP_EDEVICE when the array's address cannot be
 * obtained.  Every call on a device uses that device's one array: calls that overlap on one
 * device (other streams or host threads) race and must be serialised by the caller.  Nothing
 * in the array needs to start at zero; its contents after a call are scratch.
 */
ctp_status ctp_project_static(const ctp_plan *plan, const void *vol, ctp_dtype vol_dtype,
                              void *sino, ctp_dtype sino_dtype, int64_t batch, int accumulate,
                              hipStream_t stream);

/*
 * Back projection (Eq. 2), the exact transpose of ctp_project with the same weights:
 * vol = A^T sino, or vol += A^T sino when accumulate != 0.  Arguments as for ctp_project,
 * with the workspace sized by ctp_workspace_bytes(plan, CTP_BACKWARD, vol_dtype, sino_dtype,
 * batch).
 */
ctp_status ctp_backproject(const ctp_plan *plan, const void *sino, ctp_dtype sino_dtype,
                           void *vol, ctp_dtype vol_dtype, int64_t batch, int accumulate,
                           void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Discrete ramp filter of filtered back projection (Section 2.1; fan-beam and FDK weighting of
 * a full circular scan with uniformly spaced views, dbeta = 2 pi / n_views), applied to every
 * detector row of `batch` sinograms of the plan's geometry (any method or mode):
 *   flat:   q_i = dbeta (M du / 2) sum_k h_du(i - k) c_k p_k,   M = SDD / SAD,
 *           c_k = SDD / sqrt(SDD^2 + (u_k - x_src)^2 + (v_j - z_src)^2)   (2D: no v term);
 *   curved: q_i = dbeta (dg / (2 SAD)) sum_k (g_ik / sin g_ik)^2 h_dg(i - k) c_k p_k,
 *           dg = du / SDD, g_ik = (i - k) dg,  c_k = cos(u_k / SDD) SDD / sqrt(SDD^2 + (v_j - z_src)^2);
 * with h_a the band-limited ramp sampled at pitch a: Ram-Lak h(0) = 1/(4a^2), h(n) = 0 for even
 * n, -1/(n pi a)^2 for odd n; Shepp-Logan h(n) = -2 / (pi^2 a^2 (4n^2 - 1)).  The back
 * projection of q by a RECON-mode plan is the FBP (2D) / FDK (3D) reconstruction.
 * sino / out: device pointers in the sinogram layout; out may equal sino when the storage types
 * agree (rows are filtered in place).  FP32 arithmetic.  Asynchronous on `stream`.
 * Errors: CTP_EINVAL (NULL pointers, batch < 1, unknown dtype or window, partial overlap or
 * in-place with different types, plan of another device), CTP_EUNSUPPORTED (non-circular scan,
 * more than 5120 detector columns or 65535 views), CTP_EDEVICE (launch).
 */
ctp_status ctp_ramp_filter(const ctp_plan *plan, const void *sino, ctp_dtype sino_dtype, void *out,
                           ctp_dtype out_dtype, int64_t batch, ctp_window window,
                           hipStream_t stream);

/* Static description of a status code (error reporting of the C boundary; no computation). */
const char *ctp_status_string(ctp_status status);

/* Thread-local detail message of the last failing call on this thread ("" if none; error
 * reporting of the C boundary, no computation). */
const char *ctp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CTPROJ_H */
