// engine.h -- internal types shared by the host plan (plan.cpp) and the kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include <string>

#include "../../include/ctproj.h"

namespace ctp {

// Error reporting and plan access shared by the ABI entry points (plan.cpp).
ctp_status set_error(ctp_status st, const std::string &msg);
void clear_error();
int plan_device(const ctp_plan *plan);
// Voxel-view updates of one batch item of a call with this plan (n_vox x n_views): the serving
// engine's estimate of a request's work.
double plan_work(const ctp_plan *plan);

enum Geom : int { kFan2D = 0, kCirc = 1, kNonCirc = 2 };
enum Det : int { kFlat = 0, kCurved = 1 };
// kSFR: the SF footprint in "recon" mode (normalised to unit sum, weighted by (SAD/W)^2; the
// back projection of FBP / FDK and its transpose).
enum Method : int { kSF = 0, kDD = 1, kSFR = 2 };

#ifndef CTP_STRIPW
#define CTP_STRIPW 16
#endif
constexpr int kStripW = CTP_STRIPW;  // detector columns owned by one forward work-group
#ifndef CTP_WIDE_STRIPW
#define CTP_WIDE_STRIPW 64
#endif
constexpr int kWideStripW = CTP_WIDE_STRIPW;   // the same on short detectors (circular 3D)
constexpr int kWideStripRows = 64;
constexpr int kMaxCells = 16;    // widest supported transaxial footprint (columns)
constexpr int kRowsMax = 512;    // detector rows (or 2D batch items) held in LDS at once
#ifndef CTP_ZCHUNK
#define CTP_ZCHUNK 16
#endif
constexpr int kZChunk = CTP_ZCHUNK; // voxels per lane along z in the back projector
constexpr int kTile = 8;         // 8 x 8 voxel columns per wavefront tile
constexpr int kNCRunMax = 16;    // longest non-circular column run (slices) of either direction

// Per-view constants, object-centred coordinates (the object offset is folded into the
// source and detector), FP32.  Built in FP64 on the host.  128 bytes.
struct alignas(16) ViewRec {
    float eu[3];    // detector u axis
    float ev[3];    // detector v axis
    float n[3];     // detector normal (towards the source)
    float s[3];     // source position
    float dms[3];   // detector reference point minus source
    float seu;      // s . eu
    float sev;      // s . ev
    float sn;       // s . n
    float Du;       // flat: ((s-d).n)/du      curved: SDD/du
    float Dv;       // flat: ((s-d).n)/dv      curved: SDD/dv
    float cu;       // flat: ((s-d).eu - ue0)/du   curved: -ue0/du   (column units)
    float cv;       // ((s-d).ev - ve0)/dv                           (row units)
    float ue0;      // detector u of the first column edge (mm)
    float ve0;      // detector v of the first row edge (mm)
    float sdd;      // SDD (mm)
    float sd_ev;    // (s-d).ev (mm)
    int ydrv;       // DD: 1 = planes y = const, 0 = planes x = const
    float ddC;      // DD axial constant: -((d-s).z + ve0)/dv (row units)
    float sad;      // nominal source-to-axis distance (mm): FBP weights and ramp-filter scale
    float pad[3];
};
static_assert(sizeof(ViewRec) == 128, "ViewRec must stay 128 bytes");

// Launch-time constants shared by all kernels.
struct Params {
    int nx, ny, nz;          // volume; for 2D nz = number of batch items (see below)
    float dx, dy, dz;
    float x0, y0, z0;        // centre of voxel 0 along each axis (object-centred)
    int nu, nv;              // detector; for 2D nv = number of batch items
    float du, dv;
    int n_views;
    // Addressing.  For 3D "z" is the slice and "row" the detector row; for 2D both are the
    // batch item (the batch is processed as the axial dimension, weight 1).
    int64_t vol_z_stride;    // elements between consecutive z in the user volume
    int64_t vol_b_stride;    // elements between batch items in the user volume (3D)
    int64_t sino_row_stride; // elements between consecutive rows
    int64_t sino_view_stride;
    int64_t sino_b_stride;   // elements between batch items (3D)
    float eps;               // ramps narrower than this (cells) are steps
    int nc_runs;             // non-circular SF: column runs allowed (see the plan's bound)
    // views [v_begin, v_begin + v_count) of a forward or back projection launch (a call may
    // be split into several launches over consecutive view ranges); 0, n_views for a whole call
    int v_begin, v_count;
    // 3D: some view projects part of the volume beyond the detector rows (the back projection
    // then tests each chunk for faces that miss them all)
    int row_clip;
    // forward: detector columns per work-group strip (kStripW; kWideStripW for circular 3D
    // scans on detectors of at most kWideStripRows rows, footprints of at most 4 cells)
    int strip_w;
};

// Kernel launchers (kernels.hip).  Return hipSuccess or the launch error.
struct LaunchCfg {
    int geom, det, method, kcells;
    int n_strips, n_row_chunks;
    float acc_bound;   // bound on a detector cell's pre-amplitude sum per unit |x|
};

// Per-item fixed-point scale of the forward projector.  dtype: 0 = FP32, 1 = BF16, 2 = FP16
// (storage type of the input / output buffer).  An item is a contiguous span of item_elems
// elements; blockmax holds item_max_blocks(item_elems) floats per item, qscale two per item.
int item_max_blocks(int64_t item_elems);
hipError_t launch_item_max(const void *vol, int dtype, int64_t n_items, int64_t item_elems,
                           float *blockmax, hipStream_t st);
hipError_t launch_qscale(const float *blockmax, int64_t n_items, int bpi, float bound,
                         float *qscale, hipStream_t st);
// z-fastest FP32 copy of `batch` volumes of nz x plane, scaled by the item's 2^S (item = b, or
// item = z when item_is_z).
hipError_t launch_transpose_zfast(const void *vol, int dtype, float *volT, const float *qscale,
                                  int64_t batch, int64_t nz, int64_t plane, int item_is_z,
                                  hipStream_t st);
hipError_t launch_store_convert(const float *src, void *dst, int dtype, int64_t n, int accumulate,
                                hipStream_t st);
hipError_t launch_amp_scale(const Params &p, const LaunchCfg &c, const ViewRec *views,
                            const void *sino, int dtype, float *out, int64_t batch, hipStream_t st);
hipError_t launch_forward(const Params &p, const LaunchCfg &c, const ViewRec *views,
                          const float *volT, const float *qscale, float *sino, int64_t batch,
                          int accumulate, hipStream_t st);
// accumulate: 0 = vol = the gather, 1 = vol += the gather, 2 = the gather continues the sums
// that vol holds (the view loop starts from them: a call split into launches over consecutive
// view ranges, the later ones with 2, gives the bits of the single launch).
hipError_t launch_backward(const Params &p, const LaunchCfg &c, const ViewRec *views,
                           const float *ysc, float *vol, int64_t batch, int accumulate,
                           hipStream_t st);
// Forward / back projection of a call (accumulate = 0) split into launches of at most
// views_per_launch consecutive views, with the checks and workspace of ctp_project /
// ctp_backproject: the same bits as the single-launch call.  The serving engine uses the split
// to bound how long one of its launches holds the device.
ctp_status project_sliced(const ctp_plan *plan, const void *vol, ctp_dtype vol_dtype, void *sino,
                          ctp_dtype sino_dtype, int64_t batch, void *workspace,
                          size_t workspace_bytes, int views_per_launch, hipStream_t stream);
ctp_status backproject_sliced(const ctp_plan *plan, const void *sino, ctp_dtype sino_dtype,
                              void *vol, ctp_dtype vol_dtype, int64_t batch, void *workspace,
                              size_t workspace_bytes, int views_per_launch, hipStream_t stream);
int plan_views(const ctp_plan *plan);

// Device address of this device's copy of the library's static scratch array (looked up once
// per device, then cached), kStaticScratchBytes long: the workspace of ctp_project_static.
constexpr size_t kStaticScratchBytes = (size_t)96 << 20;
hipError_t static_scratch(void **ptr);
// Cosine-weighted ramp filter of every detector row (circular scans).  window: 0 = Ram-Lak,
// 1 = Shepp-Logan; dbeta: angular step of the scan; in / out storage types as above (in and
// out may be the same buffer when their types agree).
hipError_t launch_ramp(const Params &p, const LaunchCfg &c, const ViewRec *views, const void *in,
                       int in_dtype, void *out, int out_dtype, int64_t batch, int window,
                       float dbeta, hipStream_t st);

}  // namespace ctp
