// kernels.hip -- gfx950 kernels of the SF / DD projector pair (paper, Section 2.3).
//
// Forward (y = A x, Eq. 1) is output-stationary: a work-group owns one view and a strip of
// detector columns (kStripW; kWideStripW on short detectors), accumulates every row of that
// strip in LDS, and walks only the voxel columns whose transaxial footprint meets the strip
// (tile culling, then per-column test).  Inside a wavefront the lanes run along z of one
// voxel column (or, 32 or 16 lanes each, of two or four), so a column's transaxial footprint
// is computed once and shared by its lanes, the axial footprints of neighbouring lanes land
// in different detector rows (few LDS-atomic collisions), and the volume, read from a
// z-fastest copy, is read with unit stride.  Each strip is written once: no global atomics.
//
// Back projection (x = A^T y, Eq. 2) is voxel-stationary: each lane owns one voxel column
// and kZChunk voxels along z, loops over all views and gathers the sinogram cells its
// footprint touches (the 64 lanes of a wavefront are an 8 x 8 column tile, so their reads hit
// a few neighbouring cache lines); each voxel is written once.  It reads a copy of the
// sinogram pre-multiplied by the per-cell amplitude, which is the transpose of the forward
// pass's final per-cell scaling.
//
// Both directions call the same device functions for the footprint weights, so the pair is
// matched up to the order of the FP32 sums.
//
// A launch covers the views [v_begin, v_begin + v_count) of its call: a call may be split
// into launches over consecutive view ranges (the serving engine bounds how long one launch
// holds the device).  Forward: each view's cells belong to that view's work-groups alone.
// Back projection: launches after the first start each voxel's sum from the value the
// previous one stored, so the split gives the single launch's bits.
#include "engine.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <map>
#include <mutex>

#ifndef CTP_FWD_FAST
#define CTP_FWD_FAST 1
#endif
#ifndef CTP_CVT_TRUNC
#define CTP_CVT_TRUNC 0
#endif
#ifndef CTP_FWD_PAIRS
#define CTP_FWD_PAIRS 1   // forward: fast columns two per wavefront in runs of 8 slices
#endif
#ifndef CTP_FWD_WAVES
#define CTP_FWD_WAVES 6   // forward, circular SF: wavefronts per SIMD the registers target
#endif
#ifndef CTP_FWD_WAVES_NC
#define CTP_FWD_WAVES_NC 4   // forward, non-circular: wavefronts per SIMD the registers target
#endif
#ifndef CTP_FWD_XCDVIEWS
#define CTP_FWD_XCDVIEWS 1   // forward: each XCD an eighth of the views of every strip
#endif
#ifndef CTP_FWD_QUADS
#define CTP_FWD_QUADS 1   // forward: before the pairs, fast columns four per wavefront (16 slices)
#endif
#ifndef CTP_FWD_ITEMS
#define CTP_FWD_ITEMS 1   // forward: (column, run) items for columns beyond the row window
#endif
#ifndef CTP_FWD_QUADS_DD
#define CTP_FWD_QUADS_DD 1   // the same for the DD forward
#endif
#ifndef CTP_FWD_LANEORD
#define CTP_FWD_LANEORD 1   // forward: tile lanes along the axis where u changes most, spaced
#endif
#ifndef CTP_BWD_ZSPREAD
#define CTP_BWD_ZSPREAD 1   // back projection: z-chunks spread over the XCDs (see bwd_kernel)
#endif
#ifndef CTP_BWD_SKIP
#define CTP_BWD_SKIP 1      // back projection: chunks whose faces miss the detector rows skip
#endif
#ifndef CTP_BWD_INSIDE_WAVE
#define CTP_BWD_INSIDE_WAVE 1   // back projection: the clamped walk for the whole wavefront
#endif
#ifndef CTP_BWD_XCDTILES
#define CTP_BWD_XCDTILES 1   // back projection: each XCD an eighth of the tiles of every chunk
#endif
#ifndef CTP_BWD_PRESKIP
#define CTP_BWD_PRESKIP 1   // back projection: a cheaper skip test before the column set-up
#endif
#ifndef CTP_BWD_FAST
#define CTP_BWD_FAST 1
#endif

namespace ctp {
namespace {

// Storage types: BF16 / FP16 are converted to FP32 on load and rounded to nearest even on
// store; all arithmetic is FP32.
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(__hip_bfloat16 v) { return __bfloat162float(v); }
__device__ __forceinline__ float to_f32(__half v) { return __half2float(v); }
template <typename T> __device__ __forceinline__ T from_f32(float v);
template <> __device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ __hip_bfloat16 from_f32<__hip_bfloat16>(float v)
{
    return __float2bfloat16(v);
}
template <> __device__ __forceinline__ __half from_f32<__half>(float v) { return __float2half(v); }

// FP32 -> fixed point for the forward accumulators: round to nearest (ties upward),
// floor(x + 0.5), in one instruction (v_cvt_rpi_i32_f32; the compiler's round-to-nearest-even
// path takes two).  Unbiased, so a cell's error grows like the square root of its number of
// terms, each at most half a unit of 2^-S.  In-range inputs only (the per-item scale keeps
// every partial sum below 2^30).
__device__ __forceinline__ int to_fixed(float x)
{
#if CTP_CVT_TRUNC
    return (int)x;
#else
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
#endif
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// a / b with the hardware reciprocal (1 ulp); used where the quotient feeds a footprint
// coordinate whose FP32 rounding is already larger.
__device__ __forceinline__ float fdiv(float a, float b) { return a * fast_rcp(b); }

// atan2(y, x) of a small angle: for x > 0 and |y| < x / 64 the series r - r^3 / 3 of r = y / x,
// whose first omitted term r^5 / 5 stays below a 1e-8 part of the result (under half an FP32
// ulp); otherwise atan2f.
__device__ __forceinline__ float atan2_small(float y, float x)
{
    if (x > 0.0f && fabsf(y) < 0.015625f * x) {
        const float r = fdiv(y, x);
        return r * fmaf(-0.333333343f, r * r, 1.0f);
    }
    return atan2f(y, x);
}

__device__ __forceinline__ float readlane_f(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ int readlane_i(int v, int lane)
{
    return __builtin_amdgcn_readlane(v, lane);
}

__device__ __forceinline__ void sort4(float &a, float &b, float &c, float &d)
{
    float t;
    t = fminf(a, b); b = fmaxf(a, b); a = t;
    t = fminf(c, d); d = fmaxf(c, d); c = t;
    t = fminf(a, c); c = fmaxf(a, c); a = t;
    t = fminf(b, d); d = fmaxf(b, d); b = t;
    t = fminf(b, c); c = fmaxf(b, c); b = t;
}

// Antiderivative of the unit-height trapezoid with corners k0 <= k1 <= k2 <= k3, in detector
// cell units (cell edges are the integers).  Ramps narrower than eps are steps.
struct Trap {
    float k0, k1, k2, k3;
    float r1, rp, r2;   // rising ramp, plateau, falling ramp widths (ramps zeroed if steps)
    float h1, h2;       // 1/(2 r1), 1/(2 r2), or 0 for steps
    float area;         // G(+inf)
};

__device__ __forceinline__ Trap make_trap(float k0, float k1, float k2, float k3, float eps)
{
    Trap t;
    const float r1 = k1 - k0, r2 = k3 - k2;
    const bool s1 = r1 > eps, s2 = r2 > eps;
    t.k0 = k0;
    t.k1 = k1;
    t.k2 = k2;
    t.k3 = k3;
    t.r1 = s1 ? r1 : 0.0f;
    t.r2 = s2 ? r2 : 0.0f;
    t.rp = k2 - k1;
    t.h1 = s1 ? 0.5f * fast_rcp(r1) : 0.0f;
    t.h2 = s2 ? 0.5f * fast_rcp(r2) : 0.0f;
    t.area = 0.5f * t.r1 + t.rp + 0.5f * t.r2;
    return t;
}

__device__ __forceinline__ float trap_G(const Trap &t, float x)
{
    const float s1 = fminf(fmaxf(x - t.k0, 0.0f), t.r1);
    const float sp = fminf(fmaxf(x - t.k1, 0.0f), t.rp);
    const float s2 = fminf(fmaxf(x - t.k2, 0.0f), t.r2);
    return fmaf(s1 * s1, t.h1, sp) + fmaf(-s2 * t.h2, s2, s2);
}

// ---- transaxial footprint of a voxel column (circular scans: independent of z) ----------

// SF: u-projections of the four transaxial corners, sorted, relative to the integer column
// origin o; the amplitude l_phi0; and the axial magnification (rows per mm of z - z_src) at
// the nearest and farthest corner, which bound the axial footprint's corners (SF-TT).
struct SFCol {
    int o;
    float t0, t1, t2, t3;
    float amp;
    float An, Af;
};

template <int DET>
__device__ __forceinline__ void sf_column(const ViewRec &V, const Params &P, float xc, float yc,
                                          float zc, SFCol &c)
{
    const float hx = 0.5f * P.dx, hy = 0.5f * P.dy;
    // (p - s).eu and (s - p).n at the column centre (zc only matters for tilted poses)
    const float ac = fmaf(xc, V.eu[0], fmaf(yc, V.eu[1], fmaf(zc, V.eu[2], -V.seu)));
    const float Wc = V.sn - fmaf(xc, V.n[0], fmaf(yc, V.n[1], zc * V.n[2]));
    const float ax = hx * V.eu[0], ay = hy * V.eu[1];
    const float wx = -hx * V.n[0], wy = -hy * V.n[1];
    const float da[4] = {-ax - ay, ax - ay, -ax + ay, ax + ay};
    const float dW[4] = {-wx - wy, wx - wy, -wx + wy, wx + wy};
    float t[4], mn = 3.0e38f, mx = 0.0f, uc;
    if (DET == kFlat) {
        uc = fmaf(V.Du, fdiv(ac, Wc), V.cu);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float Wk = Wc + dW[k];
            // u_k - u_c without cancellation: Du (da W_c - a_c dW) / (W_k W_c)
            t[k] = V.Du * fdiv(fmaf(da[k], Wc, -ac * dW[k]), Wk * Wc);
            mn = fminf(mn, Wk);
            mx = fmaxf(mx, Wk);
        }
    } else {
        uc = fmaf(V.Du, atan2f(ac, Wc), V.cu);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float ak = ac + da[k], Wk = Wc + dW[k];
            // angle difference atan2(a_k, W_k) - atan2(a_c, W_c)
            t[k] = V.Du * atan2_small(fmaf(da[k], Wc, -ac * dW[k]), fmaf(Wk, Wc, ak * ac));
            const float rho2 = fmaf(ak, ak, Wk * Wk);   // squared distances: two roots below
            mn = fminf(mn, rho2);
            mx = fmaxf(mx, rho2);
        }
        mn = sqrtf(mn);
        mx = sqrtf(mx);
    }
    const float of = floorf(fminf(fmaxf(uc, -1.0e7f), 1.0e7f));
    const float base = uc - of;
    c.o = (int)of;
    c.t0 = t[0] + base;
    c.t1 = t[1] + base;
    c.t2 = t[2] + base;
    c.t3 = t[3] + base;
    sort4(c.t0, c.t1, c.t2, c.t3);
    c.An = fdiv(V.Dv, mn);
    c.Af = fdiv(V.Dv, mx);
    const float gx = xc - V.s[0], gy = yc - V.s[1];
    const float g = sqrtf(fmaf(gx, gx, gy * gy));
    c.amp = g * fminf(fdiv(P.dx, fabsf(gx)), fdiv(P.dy, fabsf(gy)));
}

// Cell weights amp * F1 for K consecutive columns starting at absolute column cs.
template <int K>
__device__ __forceinline__ void sf_cell_weights(const SFCol &c, int cs, int nc, float eps,
                                                float (&w)[K])
{
    const Trap tr = make_trap(c.t0, c.t1, c.t2, c.t3, eps);
    const float x0 = (float)(cs - c.o);
    float gprev = trap_G(tr, x0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float g = trap_G(tr, x0 + (float)(k + 1));
        w[k] = k < nc ? c.amp * (g - gprev) : 0.0f;
        gprev = g;
    }
}

// Recon mode (circular scans): amplitude (SAD / W)^2 / A_u of a voxel column, W the depth of
// the column centre (flat: along the detector normal; curved: in-plane distance from the
// source) and A_u the area of its unit-height transaxial trapezoid in columns, so that the
// column weights sum to (SAD / W)^2 on an unbounded detector.
template <int DET>
__device__ __forceinline__ float sf_recon_col_amp(const ViewRec &V, const SFCol &c, float xc,
                                                  float yc)
{
    const float Wc = V.sn - fmaf(xc, V.n[0], yc * V.n[1]);
    float W = Wc;
    if (DET == kCurved) {
        const float ac = fmaf(xc, V.eu[0], fmaf(yc, V.eu[1], -V.seu));
        W = sqrtf(fmaf(ac, ac, Wc * Wc));
    }
    const float r = fdiv(V.sad, W);
    return fdiv(r * r, 0.5f * ((c.t3 + c.t2) - (c.t1 + c.t0)));
}

// Area of an axial trapezoid in rows (exact corners; recon-mode normalisation).
__device__ __forceinline__ float trap_area(const Trap &t)
{
    return 0.5f * ((t.k3 + t.k2) - (t.k1 + t.k0));
}

// DD: columns touched by the voxel's in-plane interval on its driving plane, the fraction of
// each mapped column covered, and the axial map scale (rows per mm) along each column's
// centre ray.
template <int DET>
__device__ __forceinline__ float dd_detector_u(const ViewRec &V, float a, float W)
{
    return DET == kFlat ? fmaf(V.Du, fdiv(a, W), V.cu) : fmaf(V.Du, atan2f(a, W), V.cu);
}

template <int DET>
__device__ __forceinline__ void dd_ray_xy(const ViewRec &V, float umm, float &qx, float &qy)
{
    if (DET == kFlat) {
        qx = fmaf(umm, V.eu[0], V.dms[0]);
        qy = fmaf(umm, V.eu[1], V.dms[1]);
    } else {
        float sg, cg;
        sincosf(umm / V.sdd, &sg, &cg);
        qx = V.sdd * (sg * V.eu[0] - cg * V.n[0]);
        qy = V.sdd * (sg * V.eu[1] - cg * V.n[1]);
    }
}

template <int DET>
__device__ __forceinline__ void dd_column_range(const ViewRec &V, const Params &P, float xc,
                                                float yc, int &cmin, int &cmax)
{
    float pax, pay, pbx, pby;
    if (V.ydrv) {
        pax = xc - 0.5f * P.dx; pbx = xc + 0.5f * P.dx; pay = pby = yc;
    } else {
        pay = yc - 0.5f * P.dy; pby = yc + 0.5f * P.dy; pax = pbx = xc;
    }
    const float aa = fmaf(pax, V.eu[0], fmaf(pay, V.eu[1], -V.seu));
    const float Wa = V.sn - fmaf(pax, V.n[0], pay * V.n[1]);
    const float ab = fmaf(pbx, V.eu[0], fmaf(pby, V.eu[1], -V.seu));
    const float Wb = V.sn - fmaf(pbx, V.n[0], pby * V.n[1]);
    const float ua = dd_detector_u<DET>(V, aa, Wa), ub = dd_detector_u<DET>(V, ab, Wb);
    cmin = (int)floorf(fminf(fmaxf(fminf(ua, ub), -1.0e7f), 1.0e7f));
    cmax = (int)floorf(fminf(fmaxf(fmaxf(ua, ub), -1.0e7f), 1.0e7f));
}

template <int DET, int K>
__device__ __forceinline__ void dd_cell_weights(const ViewRec &V, const Params &P, float xc,
                                                float yc, int cs, int nc, float (&fx)[K],
                                                float (&bz)[K])
{
    const bool yd = V.ydrv != 0;
    const float plane = yd ? yc : xc;
    const float sa = yd ? V.s[1] : V.s[0], sb = yd ? V.s[0] : V.s[1];
    const float lo = yd ? xc - 0.5f * P.dx : yc - 0.5f * P.dy;
    const float hi = yd ? xc + 0.5f * P.dx : yc + 0.5f * P.dy;
    const float dist = plane - sa;
    float qx, qy;
    dd_ray_xy<DET>(V, fmaf((float)cs, P.du, V.ue0), qx, qy);
    float Xprev = fmaf(dist, fdiv(yd ? qx : qy, yd ? qy : qx), sb);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        dd_ray_xy<DET>(V, fmaf((float)(cs + k + 1), P.du, V.ue0), qx, qy);
        const float X = fmaf(dist, fdiv(yd ? qx : qy, yd ? qy : qx), sb);
        const float mlo = fminf(X, Xprev), mhi = fmaxf(X, Xprev);
        const float ov = fminf(hi, mhi) - fmaxf(lo, mlo);
        fx[k] = (k < nc && ov > 0.0f) ? fdiv(ov, mhi - mlo) : 0.0f;
        Xprev = X;
        dd_ray_xy<DET>(V, fmaf((float)cs + (float)k + 0.5f, P.du, V.ue0), qx, qy);
        bz[k] = fdiv(yd ? qy : qx, dist * P.dv);
    }
}

// ---- per-cell amplitude (applied after the forward sum / before the adjoint gather) ------

template <int GEOM, int DET, int METHOD>
__device__ __forceinline__ float cell_amp(const ViewRec &V, const Params &P, int i, int j)
{
    if (METHOD == kSFR || (GEOM == kFan2D && METHOD == kSF))
        return 1.0f;
    const float u = fmaf((float)i + 0.5f, P.du, V.ue0);
    const float v = GEOM == kFan2D ? 0.0f : fmaf((float)j + 0.5f, P.dv, V.ve0);
    float rx, ry, rz;
    if (DET == kFlat) {
        rx = fmaf(u, V.eu[0], fmaf(v, V.ev[0], V.dms[0]));
        ry = fmaf(u, V.eu[1], fmaf(v, V.ev[1], V.dms[1]));
        rz = fmaf(u, V.eu[2], fmaf(v, V.ev[2], V.dms[2]));
    } else {
        float sg, cg;
        sincosf(u / V.sdd, &sg, &cg);
        const float h = GEOM == kFan2D ? 0.0f : v - V.sd_ev;
        rx = fmaf(V.sdd, sg * V.eu[0] - cg * V.n[0], h * V.ev[0]);
        ry = fmaf(V.sdd, sg * V.eu[1] - cg * V.n[1], h * V.ev[1]);
        rz = fmaf(V.sdd, sg * V.eu[2] - cg * V.n[2], h * V.ev[2]);
    }
    if (GEOM == kFan2D)
        rz = 0.0f;
    const float r = sqrtf(fmaf(rx, rx, fmaf(ry, ry, rz * rz)));
    if (METHOD == kSF)
        return r / sqrtf(fmaf(rx, rx, ry * ry));
    return V.ydrv ? P.dy * r / fabsf(ry) : P.dx * r / fabsf(rx);
}

// ---- SF axial footprint of one voxel (circular scans) -----------------------------------

// Rows are relative to the caller's row origin; `an`, `bn`, `af`, `bf` give the v-projection
// (rows) of the voxel's bottom face at the nearest / farthest corner as a + b * z; the top
// face is one slice higher.
__device__ __forceinline__ Trap sf_axial(float an, float bn, float af, float bf, float z,
                                         float eps)
{
    const float vbn = fmaf(bn, z, an), vbf = fmaf(bf, z, af);
    const float vtn = vbn + bn, vtf = vbf + bf;
    const float k0 = fminf(vbn, vbf), k3 = fmaxf(vtn, vtf);
    const float m1 = fmaxf(vbn, vbf), m2 = fminf(vtn, vtf);
    return make_trap(k0, fminf(m1, m2), fmaxf(m1, m2), k3, eps);
}

// Visit the rows of trapezoid tr that lie in [0, R): fn(j, F_j) with F_j = G(j+1) - G(j).
// The loop is bounded by R whatever the trapezoid's position.
template <typename Fn>
__device__ __forceinline__ void for_rows(const Trap &tr, int R, Fn &&fn)
{
    const float fr = (float)R;
    const int j0 = (int)floorf(fminf(fmaxf(tr.k0, -1.0f), fr));
    const int j1 = (int)floorf(fminf(fmaxf(tr.k3, -1.0f), fr));
    const int js = max(j0, 0), je = min(j1, R - 1);
    float gprev = js > j0 ? trap_G(tr, (float)js) : 0.0f;
    for (int j = js; j <= je; ++j) {
        const float g = j < j1 ? trap_G(tr, (float)(j + 1)) : tr.area;
        fn(j, g - gprev);
        gprev = g;
    }
}

// DD axial overlap: rows j in [0, R) met by the mapped voxel interval [zl, zh] (row units);
// fn(j, overlap).
template <typename Fn>
__device__ __forceinline__ void for_dd_rows(float zl, float zh, int R, Fn &&fn)
{
    const float fr = (float)R;
    const int js = max((int)floorf(fminf(fmaxf(zl, -1.0f), fr)), 0);
    const int je = min((int)floorf(fminf(fmaxf(zh, -1.0f), fr)), R - 1);
    for (int j = js; j <= je; ++j) {
        const float wz = fminf(zh, (float)(j + 1)) - fmaxf(zl, (float)j);
        if (wz > 0.0f)
            fn(j, wz);
    }
}

// SF footprint of one voxel for non-circular poses (flat detector): everything per voxel.
struct SFVox {
    int o;              // column origin
    float t0, t1, t2, t3;
    Trap ax;            // axial trapezoid in rows relative to the row origin
};

__device__ __forceinline__ void sf_voxel_noncirc(const ViewRec &V, const Params &P, float xc,
                                                 float yc, float zc, float row0, SFVox &r)
{
    const float hx = 0.5f * P.dx, hy = 0.5f * P.dy, hz = 0.5f * P.dz;
    const float ac = fmaf(xc, V.eu[0], fmaf(yc, V.eu[1], fmaf(zc, V.eu[2], -V.seu)));
    const float Wc = V.sn - fmaf(xc, V.n[0], fmaf(yc, V.n[1], zc * V.n[2]));
    const float ax = hx * V.eu[0], ay = hy * V.eu[1];
    const float wx = -hx * V.n[0], wy = -hy * V.n[1];
    const float da[4] = {-ax - ay, ax - ay, -ax + ay, ax + ay};
    const float dW[4] = {-wx - wy, wx - wy, -wx + wy, wx + wy};
    const float iWc = fast_rcp(Wc);
    const float uc = fmaf(V.Du * ac, iWc, V.cu);
    // per transaxial corner k: depths at the mid-plane (Wk), bottom (Wb) and top (Wt) corners;
    // their three reciprocals come from one reciprocal of the product
    const float hc = fmaf(xc, V.ev[0], fmaf(yc, V.ev[1], fmaf(zc, V.ev[2], -V.sev)));
    const float ex = hx * V.ev[0], ey = hy * V.ev[1], ez = hz * V.ev[2];
    const float nzh = hz * V.n[2];
    const float dh[4] = {-ex - ey, ex - ey, -ex + ey, ex + ey};
    float t[4], vb[4], vt[4];
    const float cvr = V.cv - row0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float Wk = Wc + dW[k], Wb = Wk + nzh, Wt = Wk - nzh;
        const float bt = Wb * Wt, r3 = fast_rcp(bt * Wk);
        const float iWk = bt * r3, iWb = (Wt * Wk) * r3, iWt = (Wb * Wk) * r3;
        t[k] = V.Du * fmaf(da[k], Wc, -ac * dW[k]) * (iWk * iWc);
        vb[k] = fmaf(V.Dv * (hc + dh[k] - ez), iWb, cvr);
        vt[k] = fmaf(V.Dv * (hc + dh[k] + ez), iWt, cvr);
    }
    const float of = floorf(fminf(fmaxf(uc, -1.0e7f), 1.0e7f)), base = uc - of;
    r.o = (int)of;
    r.t0 = t[0] + base;
    r.t1 = t[1] + base;
    r.t2 = t[2] + base;
    r.t3 = t[3] + base;
    sort4(r.t0, r.t1, r.t2, r.t3);
    // axial: v of the four bottom and four top corners
    float bmn = 3.0e38f, bmx = -3.0e38f, tmn = 3.0e38f, tmx = -3.0e38f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        bmn = fminf(bmn, vb[k]);
        bmx = fmaxf(bmx, vb[k]);
        tmn = fminf(tmn, vt[k]);
        tmx = fmaxf(tmx, vt[k]);
    }
    float k0 = bmn, k1 = bmx, k2 = tmn, k3 = tmx;
    sort4(k0, k1, k2, k3);
    r.ax = make_trap(k0, k1, k2, k3, P.eps);
}

__device__ __forceinline__ float sf_amp(const ViewRec &V, const Params &P, float xc, float yc)
{
    const float gx = xc - V.s[0], gy = yc - V.s[1];
    const float g = sqrtf(fmaf(gx, gx, gy * gy));
    return g * fminf(fdiv(P.dx, fabsf(gx)), fdiv(P.dy, fabsf(gy)));
}

// ---- non-circular SF (flat detector): voxel-column runs -----------------------------------
//
// A tilted pose gives the detector axes z components, so along a voxel column the transaxial
// corners (taken at each voxel's mid-plane) drift in u and the corners of one face lie at
// different depths.  Along a column every corner's projection is a ratio of affine functions
// of the slice (or face) index j, f(j) = (N0 + a j) / (D0 + b j) = f0 + s j / (1 + r j) with
// s = (a - f0 b) / D0 and r = b / D0.  Within a run of slices it is evaluated as the
// second-order expansion f0 + s j + c j^2, c = -s r, whose remainder |s| r^2 j^3 the plan
// bounds (below 2e-5 cells or rows, else this path is off and every voxel is evaluated on its
// own).  The difference of two corners' projections has a numerator affine in j, so two
// corners change order at most once along a column: when the sorted order of the transaxial
// corners, and the two corners that bound the faces' v-intervals, agree at both ends of the
// column, they hold for all of it (otherwise the column takes the per-voxel path).

// Slopes per slice of a view's projection numerators and depths.
struct NCView {
    float aU;   // Du dz eu_z: numerator of u (columns x mm)
    float aV;   // Dv dz ev_z: numerator of v (rows x mm)
    float bW;   // -dz n_z:    depth (mm)
};

__device__ __forceinline__ NCView nc_view(const ViewRec &V, const Params &P)
{
    NCView w;
    w.aU = V.Du * P.dz * V.eu[2];
    w.aV = V.Dv * P.dz * V.ev[2];
    w.bW = -P.dz * V.n[2];
    return w;
}

// f0, s, c of f(j) = (N0 + a j) / (D0 + b j) about j = 0 (see above).
__device__ __forceinline__ void nc_expand(float N0, float D0, float a, float b, float &f0,
                                          float &s, float &c)
{
    const float iD = fast_rcp(D0);
    f0 = N0 * iD;
    s = fmaf(-f0, b, a) * iD;
    c = -s * (b * iD);
}

// A voxel column in one view.  NU, DU: numerators Du (a_c + da_k) and depths W_c + dW_k of the
// four transaxial corners at the centre of slice 0, sorted by u; NV: numerators Dv (h + dh_k) of
// the same corners at face 0 (the bottom of slice 0), whose depths are DU - bW / 2.  A face's
// v-interval is the minimum and maximum of its four corners (which corners those are changes
// along the column: near and far swap at the detector's central plane).  ok: the transaxial
// order holds along the column, every depth is positive and the faces are increasing and
// disjoint (voxel z's axial trapezoid rises over face z and falls over face z + 1); inside:
// every face lies within rows [0, R - 1) of the row window.
struct NCCol {
    float NU[4], DU[4], NV[4];
    bool ok, inside;
    int r_lo, r_hi;   // runs whose footprints may meet the strip (r_lo > r_hi: none)
};

// v-interval [p, q] (rows, without cv) of face f of a column (corners NV, DU as in NCCol).
__device__ __forceinline__ void nc_face(const float (&NV)[4], const float (&DU)[4],
                                        const NCView &w, float f, float &p, float &q)
{
    p = 3.0e38f;
    q = -3.0e38f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float v = fdiv(fmaf(f, w.aV, NV[k]), fmaf(f, w.bW, fmaf(-0.5f, w.bW, DU[k])));
        p = fminf(p, v);
        q = fmaxf(q, v);
    }
}

// nf: the faces the runs walk (the slices rounded up to whole runs of NS); cvr: V.cv minus the
// row window's first row; R: rows in the window; [ulo, uhi]: the strip's columns (absolute,
// with a margin), against which the runs are selected.
template <int NS>
__device__ __forceinline__ void nc_column(const ViewRec &V, const Params &P, const NCView &w,
                                          float xc, float yc, float cvr, int R, int nf,
                                          float ulo, float uhi, NCCol &c)
{
    const float hx = 0.5f * P.dx, hy = 0.5f * P.dy;
    const float A0 = fmaf(xc, V.eu[0], fmaf(yc, V.eu[1], fmaf(P.z0, V.eu[2], -V.seu)));
    const float W0 = V.sn - fmaf(xc, V.n[0], fmaf(yc, V.n[1], P.z0 * V.n[2]));
    const float Hf = fmaf(xc, V.ev[0], fmaf(yc, V.ev[1], fmaf(P.z0 - 0.5f * P.dz, V.ev[2], -V.sev)));
    const float zl = (float)(P.nz - 1), fl = (float)nf;
    float k0[4], k1[4];
    float dmin = 3.0e38f;      // smallest corner depth over the faces walked (affine in z)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float sx = (k & 1) ? hx : -hx, sy = (k & 2) ? hy : -hy;
        const float dW = fmaf(sx, V.n[0], sy * V.n[1]);
        c.NU[k] = V.Du * fmaf(sx, V.eu[0], fmaf(sy, V.eu[1], A0));
        c.DU[k] = W0 - dW;
        c.NV[k] = V.Dv * fmaf(sx, V.ev[0], fmaf(sy, V.ev[1], Hf));
        const float df = fmaf(-0.5f, w.bW, c.DU[k]);
        dmin = fminf(dmin, fminf(df, fmaf(fl, w.bW, df)));
        k0[k] = fdiv(c.NU[k], c.DU[k]);
        k1[k] = fdiv(fmaf(zl, w.aU, c.NU[k]), fmaf(zl, w.bW, c.DU[k]));
    }
    // transaxial corners sorted by u at slice 0, carrying their u at the last slice
    auto ce = [&](int i, int j) {
        const bool sw = k0[j] < k0[i];
        const float a0 = k0[i], a1 = k1[i], a2 = c.NU[i], a3 = c.DU[i], a4 = c.NV[i];
        k0[i] = sw ? k0[j] : a0; k0[j] = sw ? a0 : k0[j];
        k1[i] = sw ? k1[j] : a1; k1[j] = sw ? a1 : k1[j];
        c.NU[i] = sw ? c.NU[j] : a2; c.NU[j] = sw ? a2 : c.NU[j];
        c.DU[i] = sw ? c.DU[j] : a3; c.DU[j] = sw ? a3 : c.DU[j];
        c.NV[i] = sw ? c.NV[j] : a4; c.NV[j] = sw ? a4 : c.NV[j];
    };
    ce(0, 1); ce(2, 3); ce(0, 2); ce(1, 3); ce(1, 2);
    const bool tstable = k1[0] <= k1[1] && k1[1] <= k1[2] && k1[2] <= k1[3];
    // faces increasing and disjoint: p(f + 1) - q(f) at both ends (rows)
    float p0, q0, p1, q1, pl, ql, pn, qn;
    nc_face(c.NV, c.DU, w, 0.0f, p0, q0);
    nc_face(c.NV, c.DU, w, 1.0f, p1, q1);
    nc_face(c.NV, c.DU, w, fl - 1.0f, pl, ql);
    nc_face(c.NV, c.DU, w, fl, pn, qn);
    const float m = 1e-4f;
    c.ok = dmin > 0.0f && tstable && p1 - q0 >= m && pn - ql >= m;
    c.inside = p0 + cvr >= 0.0f && qn + cvr < (float)(R - 1);
    // Runs that can meet the strip: the footprint's ends t0, t3 are close to affine along the
    // column (the second-order term stays below a few hundredths of a cell over a column), so
    // the slices where [t0, t3] overlaps [ulo, uhi] (widened by 0.25 cells) form one interval.
    // Each run still tests its own cells exactly.
    const float zlast = zl > 0.0f ? zl : 1.0f;
    const float lo0 = k0[0] + V.cu, lo1 = k1[0] + V.cu, hi0 = k0[3] + V.cu, hi1 = k1[3] + V.cu;
    const float a = ulo - 0.25f, b = uhi + 0.25f;
    // z with hi(z) >= a and lo(z) <= b, hi and lo linear between slice 0 and slice zl
    float zmin = 0.0f, zmax = zl;
    const float dh = (hi1 - hi0) / zlast, dl = (lo1 - lo0) / zlast;
    if (dh > 0.0f) zmin = fmaxf(zmin, (a - hi0) / dh);
    else if (dh < 0.0f) zmax = fminf(zmax, (a - hi0) / dh);
    else if (hi0 < a) zmax = -1.0f;
    if (dl > 0.0f) zmax = fminf(zmax, (b - lo0) / dl);
    else if (dl < 0.0f) zmin = fmaxf(zmin, (b - lo0) / dl);
    else if (lo0 > b) zmax = -1.0f;
    const int nrun = nf / NS;
    if (!(zmin <= zmax)) {
        c.r_lo = 0;
        c.r_hi = -1;
    } else {
        c.r_lo = max((int)floorf(zmin / (float)NS) - 1, 0);
        c.r_hi = min((int)floorf(zmax / (float)NS) + 1, nrun - 1);
    }
}

// Slot weights of one voxel of a run: its transaxial corners t_k (columns relative to the run's
// first cell, sorted; T0_k + j (s_k + j c_k) for the run's j-th voxel), the unit-height
// trapezoid's cell
// averages F1 over the K cells from floor(t0) (its width is below K - 1 cells), times val, in
// the slots 0 .. K of the run's cells (floor(t0) is 0 or 1: the run's corners drift by less
// than a cell).
template <int K>
__device__ __forceinline__ void nc_slot_weights(const float (&t)[4], float val, float eps,
                                                float (&wv)[K + 1])
{
    // a ramp narrower than eps is a step: with the width floored at eps its quadratic part
    // a^2 / (2 max(r, eps)) (a <= r) differs from the step's by less than eps / 2
    const float r1 = t[1] - t[0], r2 = t[3] - t[2];
    const float rp = fmaxf(t[2] - t[1], 0.0f);
    const float h1 = 0.5f * fast_rcp(fmaxf(r1, eps)), h2 = 0.5f * fast_rcp(fmaxf(r2, eps));
    const float area = fmaf(0.5f, r1 + r2, rp);
    const float e0 = floorf(fmaxf(t[0], 0.0f));
    float G[K - 1];
#pragma unroll
    for (int q = 0; q < K - 1; ++q) {
        const float x = e0 + (float)(q + 1);
        const float a = __builtin_amdgcn_fmed3f(x - t[0], 0.0f, r1);
        const float b = __builtin_amdgcn_fmed3f(x - t[1], 0.0f, rp);
        const float d = __builtin_amdgcn_fmed3f(x - t[2], 0.0f, r2);
        G[q] = fmaf(a * a, h1, b) + fmaf(-d * h2, d, d);
    }
    float wc[K];
    wc[0] = G[0];
#pragma unroll
    for (int q = 1; q < K - 1; ++q)
        wc[q] = G[q] - G[q - 1];
    wc[K - 1] = area - G[K - 2];
    const bool sh = e0 >= 1.0f;
#pragma unroll
    for (int q = 0; q <= K; ++q) {
        const float lo = q >= 1 ? wc[q - 1] : 0.0f, hi = q < K ? wc[q] : 0.0f;
        wv[q] = val * (sh ? lo : hi);
    }
}

// Forward run of slices z0 .. z0 + NS - 1 of one column of a non-circular scan: as sf_fwd_run
// (running axial integral, one emit per row), with per-voxel transaxial weights, so each row
// emits K + 1 slot values, one per cell of the run (cells c_lo .. c_lo + K; the run's corners
// drift by less than one cell).  Face g's interval is [min, max] of its four corners, each
// expanded as V0 + g (Vs + g Vc) in rows relative to the run's base row edge.  acc0: LDS
// accumulator of cell c_lo in row 0 (the row has K columns of padding on both sides of the
// strip, so slots past the strip need no test).  Slices past nz continue on the same lines with
// zero values (the column tests cover faces up to nz rounded up to NS).
template <int K, bool INSIDE, int NS>
__device__ __forceinline__ void nc_fwd_walk(const float (&v)[NS], const float (&T0)[4],
                                            const float (&ts)[4], const float (&tc)[4],
                                            const float (&V0)[4], const float (&Vs)[4],
                                            const float (&Vc)[4], float base, float eps,
                                            int *acc0, int SW, int R)
{
    const float fR1 = (float)(R + 1), fRm1 = (float)(R - 1);
    // faces by second differences: x_k(g + 1) = x_k(g) + d_k(g), d_k(g + 1) = d_k(g) + 2 Vc_k
    // (the walk reaches them in order; nothing is formed ahead of time)
    float fx[4], fd[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        fx[k] = V0[k];
        fd[k] = Vs[k] + Vc[k];
    }
    auto face = [&](float &p, float &q) {
        p = fminf(fminf(fx[0], fx[1]), fminf(fx[2], fx[3]));
        q = fmaxf(fmaxf(fx[0], fx[1]), fmaxf(fx[2], fx[3]));
    };
    auto next_face = [&]() {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            fx[k] += fd[k];
            fd[k] = fmaf(2.0f, Vc[k], fd[k]);
        }
    };
    float ft = INSIDE ? 1.0f : fmaxf(base, -1.0f) + 1.0f - base;
    int *ap = acc0 - SW + __umul24((unsigned)(ft + base), SW);
    const float lim1 = fR1 - base, limm1 = fRm1 - base;
    float cp[K + 1], wvc[K + 1], wvp[K + 1];
#pragma unroll
    for (int k = 0; k <= K; ++k) {
        cp[k] = 0.0f;
        wvp[k] = 0.0f;
    }
    auto emit = [&](float al, float be) {
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            const float local = fmaf(wvc[k], al, wvp[k] * be);
            atomicAdd(ap + k, to_fixed(local - cp[k]));
            cp[k] = local;
        }
        ap += SW;
        ft += 1.0f;
    };
    float pcur, qcur;
    face(pcur, qcur);
    // transaxial corners of the current voxel by second differences, with the corners' mean
    // second-order coefficient (they differ by a relative 2 |dW| / W; the transaxial slopes are
    // small, so this moves a corner by far less than the expansion's own remainder)
    const float tc2 = 0.5f * ((tc[0] + tc[1]) + (tc[2] + tc[3]));
    float tx[4], td[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        tx[k] = T0[k];
        td[k] = ts[k] + 0.5f * tc2;
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        if (q > 0) {
#pragma unroll
            for (int k = 0; k <= K; ++k)
                wvp[k] = wvc[k];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                tx[k] += td[k];
                td[k] += tc2;
            }
        }
        nc_slot_weights<K>(tx, v[q], eps, wvc);
        next_face();
        float pn, qn;
        face(pn, qn);
        const float wq = qcur - pcur;
        const float h = 0.5f * fast_rcp(fmaxf(wq, 1e-30f));
        const float fte = INSIDE ? ceilf(pn) - 1.0f : ceilf(fminf(pn, lim1)) - 1.0f;
        // inside face q or on voxel q's plateau: with u = t - q_q, e = max(u, 0), d2 = e - u,
        // d1 = w_q - d2, local = wv_q (d1^2 / (2 w_q) + e) - wv_{q-1} d2^2 / (2 w_q)
        while (ft <= fte) {
            const float u = ft - qcur, e = fmaxf(u, 0.0f);
            const float d2 = e - u, d1 = wq - d2;
            emit(fmaf(d1 * d1, h, e), -(d2 * d2) * h);
        }
        // prefix S_{q+1} = S_q + wv_q area_q, area_q = mid_{q+1} - mid_q
        const float area = 0.5f * ((pn + qn) - (pcur + qcur));
#pragma unroll
        for (int k = 0; k <= K; ++k)
            cp[k] = fmaf(-wvc[k], area, cp[k]);
        pcur = pn;
        qcur = qn;
    }
    // above the run's top face: the last voxel's falling ramp over face NS
    {
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            wvp[k] = wvc[k];
            wvc[k] = 0.0f;
        }
        const float h = 0.5f * fast_rcp(fmaxf(qcur - pcur, 1e-30f));
        const float fte = INSIDE ? floorf(qcur) + 1.0f : floorf(fminf(qcur, limm1)) + 1.0f;
        while (ft <= fte) {
            const float d2 = fmaxf(qcur - ft, 0.0f);
            emit(0.0f, -(d2 * d2) * h);
        }
    }
}

// One run (column col_lane's slices z0 .. z0 + NS - 1) of the non-circular forward pass.
// rec: the wavefront's staged column records (rec[f][lane]: column index at 0, NU[4] at 1..,
// DU[4] at 5.., NV[4] at 9.., the amplitude at 13), read here so that they hold no registers
// during the walk.
template <int K, bool INSIDE, int NS>
__device__ __forceinline__ void nc_fwd_item(const float *__restrict__ volb, int64_t colstride,
                                            int nz, int z0, const float (*rec)[64], int src,
                                            const NCView &w, float cu, float cvr, float eps,
                                            int i_lo, int i_hi, int *acc, int SW, int R)
{
    const float fR = (float)R;
    const float z0f = (float)z0;
    // transaxial corners about slice z0, relative to the run's first cell
    float T0[4], ts[4], tc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        nc_expand(fmaf(z0f, w.aU, rec[1 + k][src]), fmaf(z0f, w.bW, rec[5 + k][src]), w.aU,
                  w.bW, T0[k], ts[k], tc[k]);
    const float o = floorf(T0[0] + cu);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        T0[k] = (T0[k] + cu) - o;
    const float jl = (float)(NS - 1);
    const float lo = fminf(T0[0], fmaf(jl, fmaf(jl, tc[0], ts[0]), T0[0]));
    const float hi = fmaxf(T0[3], fmaf(jl, fmaf(jl, tc[3], ts[3]), T0[3]));
    const float flo = floorf(lo);
    const int c_lo = (int)o + (int)flo;
    const int c_hi = (int)o + (int)floorf(hi);
    if (c_hi < i_lo || c_lo >= i_hi || c_lo < i_lo - K)
        return;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        T0[k] -= flo;
    // face corners about face z0, rows relative to the run's base row edge
    float V0[4], Vs[4], Vc[4];
    float vmin = 3.0e38f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        nc_expand(fmaf(z0f, w.aV, rec[9 + k][src]),
                  fmaf(z0f, w.bW, fmaf(-0.5f, w.bW, rec[5 + k][src])), w.aV, w.bW, V0[k], Vs[k],
                  Vc[k]);
        V0[k] += cvr;
        vmin = fminf(vmin, V0[k]);
    }
    const float base = floorf(vmin);
    float vmax = -3.0e38f;
    const float fn = (float)NS;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        V0[k] -= base;
        vmax = fmaxf(vmax, fmaf(fn, fmaf(fn, Vc[k], Vs[k]), V0[k]));
    }
    if (!INSIDE && (vmax < -base || base >= fR))
        return;
    const float amp = rec[13][src];
    const float *colp = volb + (int64_t)__float_as_int(rec[0][src]) * colstride;
    float v[NS];
    if ((nz & 3) == 0 && (NS & 3) == 0) {
#pragma unroll
        for (int g = 0; g < NS; g += 4) {
            const float4 v4 = z0 + g < nz ? *reinterpret_cast<const float4 *>(colp + z0 + g)
                                          : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            v[g] = v4.x * amp; v[g + 1] = v4.y * amp; v[g + 2] = v4.z * amp; v[g + 3] = v4.w * amp;
        }
    } else {
#pragma unroll
        for (int q = 0; q < NS; ++q)
            v[q] = z0 + q < nz ? colp[z0 + q] * amp : 0.0f;
    }
    nc_fwd_walk<K, INSIDE, NS>(v, T0, ts, tc, V0, Vs, Vc, base, eps, acc + (c_lo - i_lo), SW, R);
}

// ---- tile culling --------------------------------------------------------------------------

// Detector column range (absolute, cells) that the xy-box [x0,x1] x [y0,y1] (all z) can
// reach.  The projection of a box lies inside the hull of its projected corners.
template <int GEOM, int DET>
__device__ __forceinline__ void box_u_range(const ViewRec &V, const Params &P, float bx0,
                                            float bx1, float by0, float by1, float &umin,
                                            float &umax)
{
    umin = 3.0e38f;
    umax = -3.0e38f;
    const int nzc = GEOM == kNonCirc ? 2 : 1;
    const float zlo = P.z0 - 0.5f * P.dz, zhi = P.z0 + ((float)P.nz - 0.5f) * P.dz;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float x = (k & 1) ? bx1 : bx0, y = (k & 2) ? by1 : by0;
        for (int q = 0; q < nzc; ++q) {
            const float z = GEOM == kNonCirc ? (q ? zhi : zlo) : 0.0f;
            const float a = fmaf(x, V.eu[0], fmaf(y, V.eu[1], fmaf(z, V.eu[2], -V.seu)));
            const float W = V.sn - fmaf(x, V.n[0], fmaf(y, V.n[1], z * V.n[2]));
            const float u = DET == kFlat ? fmaf(V.Du, a / W, V.cu) : fmaf(V.Du, atan2f(a, W), V.cu);
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
        }
    }
}


// ---- forward fast path: axial resampling of one voxel column (circular SF) ----------------
//
// For a circular scan the v-projection of the face z = z_f of a voxel column is an interval
// [p_f, q_f] whose ends are affine in f (nearest / farthest corner).  When consecutive faces'
// intervals do not overlap, voxel z's SF-TT axial trapezoid rises over face z, is flat up to
// face z+1 and falls over face z+1, so for any run of slices the integral of
// sum_z x_z trap_z(v) up to row edge t is
//   on voxel z's plateau:  C(t) = S_z + x_z (w_z / 2 + t - q_z)
//   inside face z:         C(t) = S_z - x_{z-1} (q_z - t)^2 / (2 w_z) + x_z (t - p_z)^2 / (2 w_z)
// (S_z: sum of x area over the run's slices below z, area_z = mid_{z+1} - mid_z, x_{z-1} = 0 at
// the run's first face, and above the run's top face C is S minus the falling ramp).  Row j
// gets C(j+1) - C(j), which equals the sum of the run's voxels' G(j+1) - G(j).  Runs are
// independent (their contributions add), so each lane takes a run of 4 slices: neighbouring
// lanes emit different rows at the same time, and no lane needs another lane's data.
// The column values arrive pre-scaled by the item's 2^S; each row's difference is rounded into
// the 32-bit fixed-point accumulators.
__device__ __forceinline__ bool sf_fast_ok(float an, float bn, float af, float bf, int nz)
{
    // faces z and z+1 disjoint for every z: an + bn z <= af + bf (z+1) and vice versa
    const float zl = (float)(nz - 1);
    const float m = 1e-4f;
    return bn > 1e-3f && bf > 1e-3f &&
           an - af - bf <= -m && fmaf(bn - bf, zl, an - af - bf) <= -m &&
           af - an - bn <= -m && fmaf(bf - bn, zl, af - an - bn) <= -m;
}

// NC: the column's number of footprint cells in this strip (weights w[0..NC-1]); the emit of
// row j (j = -1 lands in the guard row below row 0) adds round(row value x w_k) to the NC cells.
// INSIDE: the whole column projects into rows [0, R - 1) (checked per column, uniform), so the
// row loops need no clamping to the row window.
// NS: slices per lane (4: one column per wavefront, 64 runs per 256 slices; 8: two columns per
// wavefront, lanes 0-31 and 32-63 each taking 256 slices of their own column in runs of 8;
// 16: four columns, 16 lanes each, in runs of 16).  Longer runs share their set-up and the
// rows where neighbouring runs meet over more slices.
// The column parameters may be uniform or per lane.  Every lane runs NS + 1 faces: when nz is
// not a multiple of NS, the last run continues past the top slice with zero-valued slices on
// the same face lines (the callers' fast and inside tests cover faces up to nz rounded up to a
// multiple of 8; runs of 16 are used only when nz is a multiple of 16), which only adds zero
// row values.
// One run of NS slices of a column, from slice z0 (the body of sf_fwd_run, also used for the
// (column, run) items of columns that reach beyond the row window).  area: the slices' common
// trapezoid area (rows), inv_area its reciprocal (recon mode).
template <int K, int NC, bool NORM, bool INSIDE, int NS>
__device__ __forceinline__ void sf_fwd_run_at(const float *__restrict__ colp, int nz, int z0,
                                              float an, float bn, float af, float bf,
                                              float area, float inv_area, const float (&w)[K],
                                              int *accs, int SW, int R)
{
    const float fR = (float)R, fR1 = (float)(R + 1), fRm1 = (float)(R - 1);
    // faces z0 .. z0 + NS on the near and far lines, in rows relative to the run's base
    // row edge (the subtraction is exact), so the face offsets within the run and the row
    // edges are accurate to a few ulps of the run's extent rather than of the row index
    const float z0f = (float)z0;
    const float an0 = fmaf(bn, z0f, an), af0 = fmaf(bf, z0f, af);
    const float base = floorf(fminf(an0, af0));
    const float an0r = an0 - base, af0r = af0 - base;
    // faces are formed as the walk reaches them (face f: [pf(f), qf(f)]), which keeps
    // few of them live at once
    auto pf = [&](int f) {
        return f == 0 ? fminf(an0r, af0r) : fminf(fmaf((float)f, bn, an0r), fmaf((float)f, bf, af0r));
    };
    auto qff = [&](int f) {
        return f == 0 ? fmaxf(an0r, af0r) : fmaxf(fmaf((float)f, bn, an0r), fmaf((float)f, bf, af0r));
    };
    // skip runs entirely outside the row window (before loading their slices)
    if (!INSIDE && (qff(NS) < -base || base >= fR))
        return;
    float v[NS];
    if ((nz & 3) == 0) {
#pragma unroll
        for (int g = 0; g < NS; g += 4) {
            const float4 v4 = z0 + g < nz ? *reinterpret_cast<const float4 *>(colp + z0 + g)
                                          : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            v[g] = v4.x; v[g + 1] = v4.y; v[g + 2] = v4.z; v[g + 3] = v4.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < NS; ++q)
            v[q] = z0 + q < nz ? colp[z0 + q] : 0.0f;
    }
    if constexpr (NORM) {   // recon mode: each voxel's axial trapezoid normalised to unit area
#pragma unroll
        for (int q = 0; q < NS; ++q)
            v[q] *= inv_area;
    }
    // ft: the next row edge to close (relative; row base + ft - 1, row -1 being the guard
    // row), ap: that row.  cp: C at the previous edge minus the prefix S_q of the current
    // face q, so that the row value is local(t) - cp with local(t) = C(t) - S_q a sum of a
    // few small terms.
    float ft = INSIDE ? 1.0f : fmaxf(base, -1.0f) + 1.0f - base;
    int *ap = accs - SW + __umul24((unsigned)(ft + base), SW);
    const float lim1 = fR1 - base, limm1 = fRm1 - base;   // row window (relative)
    float cp = 0.0f;
    auto emit = [&](float local) {
        const float rv = local - cp;
#pragma unroll
        for (int k = 0; k < NC; ++k)
            atomicAdd(ap + k, to_fixed(rv * w[k]));
        cp = local;
        ap += SW;
        ft += 1.0f;
    };
    // Inside face q (or on voxel q's plateau above it), with u = t - q_q, e = max(u, 0),
    // d2 = e - u = max(q_q - t, 0) and d1 = w_q - d2 = min(t - p_q, w_q):
    //   local = v_q (d1^2 / (2 w_q) + e) - v_{q-1} d2^2 / (2 w_q)
    float pc = pf(0), qc = qff(0);   // current face
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const float pn = pf(q + 1);
        const float wq = qc - pc;
        const float h = 0.5f * fast_rcp(fmaxf(wq, 1e-30f));
        const float fte = INSIDE ? ceilf(pn) - 1.0f : ceilf(fminf(pn, lim1)) - 1.0f;
        if (q == 0) {   // no voxel below the run
            while (ft <= fte) {
                const float u = ft - qc, e = fmaxf(u, 0.0f);
                const float d1 = wq - (e - u);
                emit(v[0] * fmaf(d1 * d1, h, e));
            }
        } else {
            const float nvh = -v[q - 1] * h;
            while (ft <= fte) {
                const float u = ft - qc, e = fmaxf(u, 0.0f);
                const float d2 = e - u, d1 = wq - d2;
                emit(fmaf(v[q], fmaf(d1 * d1, h, e), (d2 * d2) * nvh));
            }
        }
        cp = fmaf(-v[q], area, cp);   // S_{q+1} = S_q + v_q area
        pc = pn;
        qc = qff(q + 1);
    }
    // above the run's top face: the last voxel's falling ramp over face NS
    {
        const float h = 0.5f * fast_rcp(fmaxf(qc - pc, 1e-30f));
        const float nvh = -v[NS - 1] * h;
        const float fte = INSIDE ? floorf(qc) + 1.0f : floorf(fminf(qc, limm1)) + 1.0f;
        while (ft <= fte) {
            const float d2 = fmaxf(qc - ft, 0.0f);
            emit((d2 * d2) * nvh);
        }
    }
}

template <int K, int NC, bool NORM, bool INSIDE, int NS>
__device__ __forceinline__ void sf_fwd_run(const float *__restrict__ colp, int nz, float an,
                                           float bn, float af, float bf,
                                           const float (&w)[K], int *accs, int SW, int R,
                                           int lane)
{
    static_assert(NS == 4 || NS == 8 || NS == 16, "runs of 4, 8 or 16 slices");
    // every slice's trapezoid has the same area, the distance between consecutive face centres
    const float area = 0.5f * (bn + bf);
    const float inv_area = NORM ? fast_rcp(area) : 1.0f;
    const int l = lane & (256 / NS - 1);
    for (int zb = 0; zb < nz; zb += 256) {
        const int z0 = zb + NS * l;
        if (z0 >= nz)
            break;
        sf_fwd_run_at<K, NC, NORM, INSIDE, NS>(colp, nz, z0, an, bn, af, bf, area, inv_area, w,
                                               accs, SW, R);
    }
}

// Dispatch the SF run on the column's (or column pair's) cell count, uniform across the
// wavefront.
template <int K, bool NORM, bool INSIDE, int NS>
__device__ __forceinline__ void sf_fwd_run_nc(const float *__restrict__ colp, int nz, float an,
                                              float bn, float af, float bf,
                                              const float (&w)[K], int nc, int *accs, int SW,
                                              int R, int lane)
{
    if constexpr (K <= 4) {
        switch (nc) {
        case 1: sf_fwd_run<K, 1, NORM, INSIDE, NS>(colp, nz, an, bn, af, bf, w, accs, SW, R, lane); return;
        case 2: sf_fwd_run<K, 2, NORM, INSIDE, NS>(colp, nz, an, bn, af, bf, w, accs, SW, R, lane); return;
        case 3: sf_fwd_run<K, (K >= 3 ? 3 : K), NORM, INSIDE, NS>(colp, nz, an, bn, af, bf, w, accs, SW, R, lane); return;
        default: sf_fwd_run<K, K, NORM, INSIDE, NS>(colp, nz, an, bn, af, bf, w, accs, SW, R, lane); return;
        }
    } else {
        // wide footprints: all K cells (weights past nc are zero; the extra cells stay within
        // the strip row plus its padding)
        sf_fwd_run<K, K, NORM, INSIDE, NS>(colp, nz, an, bn, af, bf, w, accs, SW, R, lane);
    }
}

// DD forward, circular: for column k of the footprint the slices' mapped z-intervals
// [zeta_z, zeta_{z+1}] (rows, zeta_z = al_k + be_k z) tile the axis, so the run's integral up to
// row edge t inside slice z is S_z + x_z (t - zeta_z) and row j gets C(j+1) - C(j) times the
// column's transaxial fraction.  Same run-per-lane scheme as the SF path.
// NS: slices per lane as in sf_fwd_run (8: two columns per wavefront, parameters per lane).
template <int K, int NS>
__device__ __forceinline__ void dd_fwd_run(const float *__restrict__ colp, int nz,
                                           const float (&al)[K], const float (&be)[K],
                                           const float (&fx)[K], int nc, int *accs,
                                           int SW, int R, int lane)
{
    // Every lane runs NS + 1 boundaries; past the top slice (nz not a multiple of NS) the run
    // continues with zero-valued slices, which only adds zero row values.
    static_assert(NS == 4 || NS == 8 || NS == 16, "runs of 4, 8 or 16 slices");
    const float fR = (float)R, fR1 = (float)(R + 1), fRm1 = (float)(R - 1);
    const int l = lane & (256 / NS - 1);
    for (int zb = 0; zb < nz; zb += 256) {
        const int z0 = zb + NS * l;
        if (z0 >= nz)
            break;
        float v[NS];
        if ((nz & 3) == 0) {
#pragma unroll
            for (int g = 0; g < NS; g += 4) {
                const float4 v4 = z0 + g < nz ? *reinterpret_cast<const float4 *>(colp + z0 + g)
                                              : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                v[g] = v4.x; v[g + 1] = v4.y; v[g + 2] = v4.z; v[g + 3] = v4.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < NS; ++q)
                v[q] = z0 + q < nz ? colp[z0 + q] : 0.0f;
        }
        const float z0f = (float)z0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k >= nc)
                break;
            // boundaries relative to the run's base row edge (exact subtraction)
            const float z00 = fmaf(be[k], z0f, al[k]);
            const float base = floorf(z00);
            const float zt0 = z00 - base;
            auto zt = [&](int f) { return f == 0 ? zt0 : fmaf((float)f, be[k], zt0); };
            if (zt(NS) < -base || base >= fR)
                continue;
            // ft: the next row edge to close (relative; row base + ft - 1, row -1 being the
            // guard row), ap: that row's cell k; cp: C at the previous edge minus the prefix of
            // the current slice
            float ft = fmaxf(base, -1.0f) + 1.0f - base;
            int *ap = accs + k - SW + __umul24((unsigned)(ft + base), SW);
            const float lim1 = fR1 - base, limm1 = fRm1 - base;
            float cp = 0.0f;
            auto emit = [&](float local) {
                atomicAdd(ap, to_fixed((local - cp) * fx[k]));
                cp = local;
                ap += SW;
                ft += 1.0f;
            };
            float zc = zt0;
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const float zn = zt(q + 1);
                const float fte = ceilf(fminf(zn, lim1)) - 1.0f;
                while (ft <= fte)
                    emit(v[q] * (ft - zc));
                cp = fmaf(-v[q], be[k], cp);     // every slice maps to be rows
                zc = zn;
            }
            const float fte = floorf(fminf(zc, limm1)) + 1.0f;
            while (ft <= fte)
                emit(0.0f);
        }
    }
}

// Non-circular SF forward: column runs of kNCRun slices for footprints of at most 4 cells
// (the run's cells then fit K + 1 slots), otherwise the per-voxel loop only.  The plan bounds
// the expansion error and the drift over runs of kNCRunMax = 16 slices.
#ifndef CTP_NC_RUN
#define CTP_NC_RUN 16
#endif
constexpr int kNCRun = CTP_NC_RUN;
static_assert(kNCRun <= kNCRunMax, "the plan bounds runs of at most kNCRunMax slices");
template <int GEOM, int METHOD, int K>
constexpr bool nc_fwd_runs() { return GEOM == kNonCirc && METHOD == kSF && K <= 4 && CTP_FWD_FAST; }
// Forward LDS row: the strip plus one padding column; the non-circular runs add K columns on
// each side.
// LDS row width of a forward strip of STW columns: its columns, one spare, and for the
// non-circular runs K padding columns on each side.
template <int GEOM, int METHOD, int K, int STW>
constexpr int fwd_row_width() { return STW + 1 + (nc_fwd_runs<GEOM, METHOD, K>() ? 2 * K : 0); }

constexpr int kListCap = 1024;
constexpr int kLaneItems = 32;   // 2D batches up to this size: each lane scatters its own pixel

// 2D forward with a small batch: lane = pixel, looping over the batch items itself (the
// broadcast scheme puts the items on the lanes, which leaves most lanes idle for a few items).
template <int K>
__device__ __forceinline__ void fan2d_lane_scatter(const float *__restrict__ colp, int zbeg,
                                                   int zend, int r0, const float (&w)[K],
                                                   int nc, int *accs, int SW)
{
    if (nc <= 0)
        return;
    for (int z = zbeg; z < zend; ++z) {
        const float val = colp[z];
        int *a = accs + (z - r0) * SW;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k < nc)
                atomicAdd(a + k, to_fixed(val * w[k]));
    }
}

// ============================================================================================
// Forward projector
// ============================================================================================
#ifndef CTP_FWD_THREADS
#define CTP_FWD_THREADS 512
#endif
constexpr int kFwdThreads = CTP_FWD_THREADS;
// Circular SF / recon-mode SF forward: 80 VGPRs for 6 wavefronts per SIMD (the LDS of three
// 512-thread work-groups per CU allows 6), with the 16-slice runs of four columns per
// wavefront; DD and non-circular keep the 128-VGPR target (measured faster or spill-free).
template <int GEOM, int METHOD>
constexpr int fwd_waves()
{
    return GEOM == kCirc && METHOD != kDD ? CTP_FWD_WAVES : GEOM == kNonCirc ? CTP_FWD_WAVES_NC : 4;
}
constexpr int kFwdWaves = kFwdThreads / 64;

// STW: detector columns per strip (kStripW, or kWideStripW on short detectors).
template <int GEOM, int DET, int METHOD, int K, int STW>
__global__ __launch_bounds__(kFwdThreads) __attribute__((amdgpu_waves_per_eu(fwd_waves<GEOM, METHOD>()))) void fwd_kernel(Params P, const ViewRec *__restrict__ views,
                                                  const float *__restrict__ volT,
                                                  const float *__restrict__ qscale,
                                                  float *__restrict__ sino, int accumulate,
                                                  int n_row_chunks)
{
    // Fixed-point accumulators: on gfx950 an LDS integer add costs a few cycles per
    // wavefront while the FP32 LDS atomic is far slower.  The z-fastest volume copy holds
    // x * 2^S with S chosen per batch item from that item's max |x| (so its strip sums fit in
    // 31 bits); contributions are converted to integers and summed, which is order
    // independent, so an item's result is bitwise repeatable and does not depend on the
    // other items of the batch.  qscale[2 b + 1] = 2^-S undoes the scale on write-out.
    extern __shared__ int acc_mem[];         // guard row, [R][SW], kMaxCells of padding
    __shared__ int s_count, s_next;
    __shared__ unsigned short s_list[kListCap];
    // 3D runs: each wavefront stages its tile's column parameters here (record field f of
    // column c at s_colrec[wave][f][c]: voxel column index, strip slot, cell count, then SF: the
    // axial lines an, bn, af, bf and the K cell weights; DD: the K overlap fractions and axial
    // map scales), so that they do not occupy registers while the columns are walked
    constexpr bool STAGE = METHOD != kDD && GEOM == kCirc && CTP_FWD_FAST;
    constexpr bool STAGE_DD = METHOD == kDD && GEOM == kCirc && CTP_FWD_FAST;
    // non-circular SF column runs (footprints of at most 4 cells): column index, NU[4], DU[4],
    // NV[4], amplitude, and per column that runs: its lane and first item, its first run
    constexpr bool STAGE_NC = nc_fwd_runs<GEOM, METHOD, K>();
    constexpr int kRecFields = STAGE ? 7 + K : STAGE_DD ? 3 + 2 * K : STAGE_NC ? 16 : 1;
    __shared__ float s_colrec[STAGE || STAGE_DD || STAGE_NC ? kFwdThreads / 64 : 1][kRecFields][64];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // XCD-aware order: work-group i runs on XCD i % 8.  XCD x takes the x-th eighth of the
    // views of every strip, strip by strip, so that the work-groups sharing an XCD's L2
    // project neighbouring views of the same strip (their voxel wedges overlap) and the XCDs
    // get equal work whatever the strip count and however the strips' work differs.  (The
    // older order, XCD x taking all views of the strips x, x + 8, ..., left the XCDs
    // unevenly loaded: 256^3 forward 5.67 -> 5.40 ms with this one, same bits.)
    const int n_strips = (P.nu + STW - 1) / STW;
    const int xcd = blockIdx.x & 7, kk = blockIdx.x >> 3;
#if CTP_FWD_XCDVIEWS
    const int vb = (P.v_count + 7) >> 3;
    if (kk >= n_strips * vb)
        return;
    const int strip = kk / vb, vl = xcd * vb + kk % vb;
    if (vl >= P.v_count)
        return;
    const int view = P.v_begin + vl;
#else
    if (kk >= ((n_strips - xcd + 7) >> 3) * P.v_count)
        return;
    const int strip = xcd + 8 * (kk / P.v_count), view = P.v_begin + kk % P.v_count;
#endif
    const int chunk = blockIdx.y % n_row_chunks;
    const int b = blockIdx.y / n_row_chunks;            // batch item (3D); 0 in 2D
    const int i_lo = strip * STW;
    const int i_hi = min(i_lo + STW, P.nu);
    const int rows_total = GEOM == kFan2D ? P.nz : P.nv;
    const int r0 = chunk * kRowsMax;
    const int R = min(kRowsMax, rows_total - r0);
    const ViewRec V = views[view];
    constexpr int SW = fwd_row_width<GEOM, METHOD, K, STW>();
    // row -1 (the guard) absorbs emits below row 0; the non-circular runs also write up to K
    // cells on either side of the strip (padding columns, never written out)
    int *acc = acc_mem + SW + (STAGE_NC ? K : 0);
    for (int e = threadIdx.x; e < (R + 1) * SW + kMaxCells; e += blockDim.x)
        acc_mem[e] = 0;

    const float hz = 0.5f * P.dz;
    const float zb0 = P.z0 - hz - V.s[2];               // bottom face of slice 0, minus z_src
    const int tiles_x = (P.nx + kTile - 1) / kTile;
    const int tiles_y = (P.ny + kTile - 1) / kTile;
    const int ntiles = tiles_x * tiles_y;
    // voxel "z" run handled by the lanes: slices (3D) or batch items in this chunk (2D)
    const int zbeg = GEOM == kFan2D ? r0 : 0;
    const int zend = GEOM == kFan2D ? r0 + R : P.nz;
    const float ulo = (float)i_lo - 1e-3f, uhi = (float)i_hi + 1e-3f;
    const int64_t colstride = P.nz;      // z-fastest copy: one voxel column is contiguous
    const float *volb = volT + (GEOM == kFan2D ? 0 : (int64_t)b * P.nx * P.ny * P.nz);

    for (int t0 = 0; t0 < ntiles; t0 += kListCap) {
        const int tend = min(t0 + kListCap, ntiles);
        if (threadIdx.x == 0) {
            s_count = 0;
            s_next = 0;
        }
        __syncthreads();
        for (int tt = t0 + wave * 64; tt < tend; tt += kFwdThreads) {
            const int t = tt + lane;
            bool hit = false;
            if (t < tend) {
                const int tx = t % tiles_x, ty = t / tiles_x;
                const float bx0 = P.x0 + ((float)(tx * kTile) - 0.5f) * P.dx;
                const float bx1 = P.x0 + ((float)min(tx * kTile + kTile, P.nx) - 0.5f) * P.dx;
                const float by0 = P.y0 + ((float)(ty * kTile) - 0.5f) * P.dy;
                const float by1 = P.y0 + ((float)min(ty * kTile + kTile, P.ny) - 0.5f) * P.dy;
                float umin, umax;
                box_u_range<GEOM, DET>(V, P, bx0, bx1, by0, by1, umin, umax);
                hit = umax >= ulo && umin <= uhi;
            }
            const uint64_t m = __ballot(hit);
            const int pre = __popcll(m & ((1ull << lane) - 1ull));
            int base = 0;
            if (lane == 0 && m)
                base = atomicAdd(&s_count, (int)__popcll(m));
            base = __shfl(base, 0);
            if (hit)
                s_list[base + pre] = (unsigned short)(t - t0);
        }
        __syncthreads();
        const int nhit = s_count;

        // waves take hit tiles from a shared counter (tiles differ in work)
        for (;;) {
            int h = 0;
            if (lane == 0)
                h = atomicAdd(&s_next, 1);
            h = __builtin_amdgcn_readfirstlane(__shfl(h, 0));
            if (h >= nhit)
                break;
            const int t = t0 + s_list[h];
            const int tx = t % tiles_x, ty = t / tiles_x;
            // lanes -> columns of the 8 x 8 tile: along the axis on which u changes most in
            // this view, every other column first (0, 2, 4, 6, 1, 3, 5, 7), so that the
            // columns walked together in one wavefront (four or two at a time, or the runs of
            // neighbouring columns) project at least ~1.4 cells apart and their same-row
            // atomics rarely meet at one LDS address (sums are integers: any order gives
            // the same bits)
            const int la = lane & (kTile - 1), lb = lane >> 3;
            const int lmaj = CTP_FWD_LANEORD ? ((la & 3) << 1) | (la >> 2) : la;
            const bool ymaj = CTP_FWD_LANEORD && fabsf(V.eu[1]) > fabsf(V.eu[0]);
            const int ix = tx * kTile + (ymaj ? lb : lmaj);
            const int iy = ty * kTile + (ymaj ? lmaj : lb);
            const bool valid = ix < P.nx && iy < P.ny;
            const float xc = fmaf((float)ix, P.dx, P.x0), yc = fmaf((float)iy, P.dy, P.y0);

            if constexpr (METHOD != kDD && GEOM != kNonCirc) {
                SFCol col;
                sf_column<DET>(V, P, xc, yc, 0.0f, col);
                if constexpr (METHOD == kSFR)
                    col.amp = sf_recon_col_amp<DET>(V, col, xc, yc);
                const int cmin = col.o + (int)floorf(col.t0), cmax = col.o + (int)floorf(col.t3);
                const int cs = max(cmin, i_lo), ce = min(cmax, i_hi - 1);
                const int nc = valid ? max(ce - cs + 1, 0) : 0;
                float w[K];
                sf_cell_weights<K>(col, cs, nc, P.eps, w);
                if constexpr (GEOM == kFan2D) {
                    if (zend - zbeg <= kLaneItems) {
                        fan2d_lane_scatter<K>(volb + ((int64_t)iy * P.nx + ix) * colstride, zbeg,
                                              zend, r0, w, nc, acc + (cs - i_lo), SW);
                        continue;
                    }
                }
                const float an = fmaf(col.An, zb0, V.cv - (float)r0), bn = col.An * P.dz;
                const float af = fmaf(col.Af, zb0, V.cv - (float)r0), bf = col.Af * P.dz;
                // each lane tests its own column for the run path (faces disjoint and
                // increasing; inside: the whole column projects into rows [0, R - 1)); the
                // broadcast loop below reads the answers from two masks
                uint64_t m_fast = 0, m_inside = 0;
                if constexpr (GEOM != kFan2D && CTP_FWD_FAST) {
                    // the runs cover faces up to nz rounded up to a multiple of 8
                    const int nz8 = (P.nz + 7) & ~7;
                    const bool fast = nc > 0 && sf_fast_ok(an, bn, af, bf, nz8);
                    const float fnz = (float)nz8;
                    const bool inside = fast && fminf(an, af) >= 0.0f &&
                                        fmaxf(fmaf(bn, fnz, an), fmaf(bf, fnz, af)) < (float)(R - 1);
                    m_fast = __ballot(fast);
                    m_inside = __ballot(inside);
                }
                float (*rec)[64] = s_colrec[STAGE || STAGE_DD ? wave : 0];
                if constexpr (STAGE) {
                    rec[0][lane] = __int_as_float(iy * P.nx + ix);
                    rec[1][lane] = __int_as_float(cs - i_lo);
                    rec[2][lane] = __int_as_float(nc);
                    rec[3][lane] = an;
                    rec[4][lane] = bn;
                    rec[5][lane] = af;
                    rec[6][lane] = bf;
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        rec[7 + k][lane] = w[k];
                }
                uint64_t m = __ballot(nc > 0);
                if constexpr (STAGE && CTP_FWD_ITEMS) {
                    if ((P.nz & 15) == 0 && (m_fast & ~m_inside) != 0) {
                        // some fast columns reach beyond the row window (a volume taller than
                        // the detector's reach): only the 16-slice runs of the fast columns
                        // whose faces can meet the window become (column, run) items, spread
                        // over the lanes (an exclusive scan of the run counts, a binary
                        // search per item); every run still tests its own rows
                        const int nrun = P.nz >> 4;
                        int rlo = 0, nr = 0;
                        if ((m_fast >> lane) & 1ull) {
                            // faces f with q(f) >= 0 start after fq, faces with p(f) < R end
                            // before fp (both lines increase); a run covers faces 16r..16r+16
                            const float fq = fminf(-an / bn, -af / bf);
                            const float fp = fmaxf(((float)R - an) / bn, ((float)R - af) / bf);
                            rlo = max((int)floorf(fmaxf(fq, -1.0e6f) * (1.0f / 16.0f)) - 2, 0);
                            const int rhi = min((int)floorf(fminf(fp, 1.0e6f) * (1.0f / 16.0f)) + 1,
                                                nrun - 1);
                            nr = max(rhi - rlo + 1, 0);
                        }
                        int incl = nr;
#pragma unroll
                        for (int d = 1; d < 64; d <<= 1) {
                            const int t = __shfl_up(incl, d);
                            if (lane >= d)
                                incl += t;
                        }
                        const int excl = incl - nr;
                        const int items = __shfl(incl, 63);
                        // the emit width: the widest fast column's cell count
                        int wnc = ((m_fast >> lane) & 1ull) ? nc : 0;
#pragma unroll
                        for (int d = 32; d >= 1; d >>= 1)
                            wnc = max(wnc, __shfl_xor(wnc, d));
                        auto run_items = [&](auto ncc) {
                            constexpr int NC = decltype(ncc)::value;
                            for (int b0 = 0; b0 < items; b0 += 64) {
                                const int it = b0 + lane;
                                // the last column whose first item is at most it: a binary
                                // search over the lanes' exclusive sums, six steps taken by
                                // every lane (the shuffles read from all lanes)
                                int src = 0;
#pragma unroll
                                for (int step = 32; step >= 1; step >>= 1) {
                                    const int mid = src + step;
                                    const int e = __shfl(excl, min(mid, 63));
                                    if (mid < 64 && e <= it)
                                        src = mid;
                                }
                                const int run = __shfl(rlo, src) + (it - __shfl(excl, src));
                                if (it < items) {
                                    float lw[K];
#pragma unroll
                                    for (int k = 0; k < K; ++k)
                                        lw[k] = rec[7 + k][src];
                                    const float l_an = rec[3][src], l_bn = rec[4][src];
                                    const float l_af = rec[5][src], l_bf = rec[6][src];
                                    const float area = 0.5f * (l_bn + l_bf);
                                    const float *colp = volb + (int64_t)__float_as_int(rec[0][src]) * colstride;
                                    sf_fwd_run_at<K, NC, METHOD == kSFR, false, 16>(
                                        colp, P.nz, 16 * run, l_an, l_bn, l_af, l_bf, area,
                                        METHOD == kSFR ? fast_rcp(area) : 1.0f, lw,
                                        acc + __float_as_int(rec[1][src]), SW, R);
                                }
                            }
                        };
                        if constexpr (K <= 4) {
                            if (wnc <= 1)
                                run_items(std::integral_constant<int, 1>{});
                            else if (wnc == 2)
                                run_items(std::integral_constant<int, (K >= 2 ? 2 : K)>{});
                            else if (wnc == 3)
                                run_items(std::integral_constant<int, (K >= 3 ? 3 : K)>{});
                            else
                                run_items(std::integral_constant<int, K>{});
                        } else {
                            run_items(std::integral_constant<int, K>{});
                        }
                        m &= ~m_fast;
                    }
                }
                if constexpr (STAGE && CTP_FWD_PAIRS) {
                    // two fast columns at a time, lanes 0-31 on the first and 32-63 on the
                    // second, each lane running 8 slices and reading its column's record
                    uint64_t mp = m & m_fast;
                    if (CTP_FWD_QUADS && (P.nz & 15) == 0) {
                        // four fast columns at a time, 16 lanes each running 16 slices
                        while (__popcll(mp) >= 4) {
                            int cq[4];
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                cq[i] = __ffsll((unsigned long long)mp) - 1;
                                mp &= mp - 1ull;
                                m &= ~(1ull << cq[i]);
                            }
                            const int src = lane < 32 ? (lane < 16 ? cq[0] : cq[1])
                                                      : (lane < 48 ? cq[2] : cq[3]);
                            const int p_nc = max(max(__float_as_int(rec[2][cq[0]]), __float_as_int(rec[2][cq[1]])),
                                                 max(__float_as_int(rec[2][cq[2]]), __float_as_int(rec[2][cq[3]])));
                            const bool p_inside = ((m_inside >> cq[0]) & (m_inside >> cq[1]) &
                                                   (m_inside >> cq[2]) & (m_inside >> cq[3]) & 1ull) != 0;
                            const int l_col = __float_as_int(rec[0][src]);
                            const int l_slot = __float_as_int(rec[1][src]);
                            float lw[K];
#pragma unroll
                            for (int k = 0; k < K; ++k)
                                lw[k] = rec[7 + k][src];
                            const float l_an = rec[3][src], l_bn = rec[4][src];
                            const float l_af = rec[5][src], l_bf = rec[6][src];
                            const float *colp = volb + (int64_t)l_col * colstride;
                            int *accs = acc + l_slot;
                            if (p_inside)
                                sf_fwd_run_nc<K, METHOD == kSFR, true, 16>(colp, P.nz, l_an, l_bn, l_af,
                                                                           l_bf, lw, p_nc, accs, SW, R,
                                                                           lane);
                            else
                                sf_fwd_run_nc<K, METHOD == kSFR, false, 16>(colp, P.nz, l_an, l_bn, l_af,
                                                                            l_bf, lw, p_nc, accs, SW, R,
                                                                            lane);
                        }
                    }
                    while (__popcll(mp) >= 2) {
                        const int c1 = __ffsll((unsigned long long)mp) - 1;
                        mp &= mp - 1ull;
                        const int c2 = __ffsll((unsigned long long)mp) - 1;
                        mp &= mp - 1ull;
                        m &= ~((1ull << c1) | (1ull << c2));
                        const int src = lane < 32 ? c1 : c2;
                        const int p_nc = max(__float_as_int(rec[2][c1]), __float_as_int(rec[2][c2]));
                        const bool p_inside = ((m_inside >> c1) & (m_inside >> c2) & 1ull) != 0;
                        const int l_col = __float_as_int(rec[0][src]);
                        const int l_slot = __float_as_int(rec[1][src]);
                        float lw[K];
#pragma unroll
                        for (int k = 0; k < K; ++k)
                            lw[k] = rec[7 + k][src];
                        const float l_an = rec[3][src], l_bn = rec[4][src];
                        const float l_af = rec[5][src], l_bf = rec[6][src];
                        const float *colp = volb + (int64_t)l_col * colstride;
                        int *accs = acc + l_slot;
                        if (p_inside)
                            sf_fwd_run_nc<K, METHOD == kSFR, true, 8>(colp, P.nz, l_an, l_bn, l_af,
                                                                      l_bf, lw, p_nc, accs, SW, R,
                                                                      lane);
                        else
                            sf_fwd_run_nc<K, METHOD == kSFR, false, 8>(colp, P.nz, l_an, l_bn, l_af,
                                                                       l_bf, lw, p_nc, accs, SW, R,
                                                                       lane);
                    }
                }
                while (m) {
                    const int c = __ffsll((unsigned long long)m) - 1;
                    m &= m - 1ull;
                    // column c's parameters as scalars (from the staged record or the lanes)
                    auto col_i = [&](int f, int v) -> int {
                        if constexpr (STAGE)
                            return __builtin_amdgcn_readfirstlane(__float_as_int(rec[f][c]));
                        else
                            return readlane_i(v, c);
                    };
                    auto col_f = [&](int f, float v) -> float {
                        if constexpr (STAGE)
                            return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(rec[f][c])));
                        else
                            return readlane_f(v, c);
                    };
                    const int s_col = col_i(0, iy * P.nx + ix);
                    const int s_slot = col_i(1, cs - i_lo), s_nc = col_i(2, nc);
                    float sw[K];
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        sw[k] = col_f(7 + k, w[k]);
                    const float s_an = col_f(3, an), s_bn = col_f(4, bn);
                    const float s_af = col_f(5, af), s_bf = col_f(6, bf);
                    const float *colp = volb + (int64_t)s_col * colstride;
                    int *accs = acc + s_slot;
                    if constexpr (GEOM != kFan2D && CTP_FWD_FAST) {
                        if ((m_fast >> c) & 1ull) {
                            if ((m_inside >> c) & 1ull)
                                sf_fwd_run_nc<K, METHOD == kSFR, true, 4>(colp, P.nz, s_an, s_bn, s_af,
                                                                       s_bf, sw, s_nc, accs, SW, R,
                                                                       lane);
                            else
                                sf_fwd_run_nc<K, METHOD == kSFR, false, 4>(colp, P.nz, s_an, s_bn, s_af,
                                                                        s_bf, sw, s_nc, accs, SW, R,
                                                                        lane);
                            continue;
                        }
                    }
                    for (int zb = zbeg; zb < zend; zb += 256) {
                        // issue the column's loads first, then compute
                        float vals[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int z = zb + lane + 64 * q;
                            vals[q] = z < zend ? colp[z] : 0.0f;
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int z = zb + lane + 64 * q;
                            if (z >= zend)
                                break;
                            const float val = vals[q];
                            if constexpr (GEOM == kFan2D) {
                                int *a = accs + (z - r0) * SW;
#pragma unroll
                                for (int k = 0; k < K; ++k)
                                    if (k < s_nc)
                                        atomicAdd(a + k, to_fixed(val * sw[k]));
                            } else {
                                const Trap tr = sf_axial(s_an, s_bn, s_af, s_bf, (float)z, P.eps);
                                const float vn = METHOD == kSFR ? fdiv(val, trap_area(tr)) : val;
                                for_rows(tr, R, [&](int j, float F) {
                                    const float f = F * vn;
                                    int *a = accs + j * SW;
#pragma unroll
                                    for (int k = 0; k < K; ++k)
                                        if (k < s_nc)
                                            atomicAdd(a + k, to_fixed(f * sw[k]));
                                });
                            }
                        }
                    }
                }
            } else if constexpr (METHOD == kSF && GEOM == kNonCirc) {
                // conservative per-column test over all z
                float umin, umax;
                box_u_range<GEOM, DET>(V, P, xc - 0.5f * P.dx, xc + 0.5f * P.dx,
                                       yc - 0.5f * P.dy, yc + 0.5f * P.dy, umin, umax);
                const bool hit = valid && umax >= ulo && umin <= uhi;
                const float amp = sf_amp(V, P, xc, yc);
                uint64_t m = __ballot(hit);
                if constexpr (STAGE_NC) {
                    if (P.nc_runs) {
                        // columns whose transaxial corner order holds and whose faces are
                        // disjoint run in runs of kNCRun slices: the (column, run) items of
                        // all such columns of the tile are spread over the lanes; the other
                        // columns take the per-voxel loop below
                        const NCView w = nc_view(V, P);
                        const int nrun = (P.nz + kNCRun - 1) / kNCRun;
                        NCCol col;
                        nc_column<kNCRun>(V, P, w, xc, yc, V.cv - (float)r0, R, nrun * kNCRun,
                                          (float)i_lo, (float)i_hi, col);
                        const bool ok = hit && col.ok;
                        const uint64_t m_ok = __ballot(ok);
                        const bool all_in = __ballot(ok && col.inside) == m_ok;
                        m &= ~m_ok;
                        float (*rec)[64] = s_colrec[wave];
                        rec[0][lane] = __int_as_float(iy * P.nx + ix);
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            rec[1 + k][lane] = col.NU[k];
                            rec[5 + k][lane] = col.DU[k];
                            rec[9 + k][lane] = col.NV[k];
                        }
                        rec[13][lane] = amp;
                        // the (column, run) items of the runs that can meet the strip: the
                        // ok columns in lane order, each with its first run and its first
                        // item (an exclusive prefix sum of the run counts over the lanes)
                        const int nr = ok ? max(col.r_hi - col.r_lo + 1, 0) : 0;
                        int incl = nr;
#pragma unroll
                        for (int d = 1; d < 64; d <<= 1) {
                            const int t = __shfl_up(incl, d);
                            if (lane >= d)
                                incl += t;
                        }
                        const int items = __shfl(incl, 63);
                        if (ok) {
                            const int j = (int)__popcll(m_ok & ((1ull << lane) - 1ull));
                            rec[14][j] = __int_as_float(lane | ((incl - nr) << 6));
                            rec[15][j] = __int_as_float(col.r_lo);
                        }
                        const int n_ok = (int)__popcll(m_ok);
                        // item it: the last ok column whose first item is at most it
                        auto item = [&](int it, int &src, int &run) {
                            int jl = 0, jh = n_ok - 1;
                            while (jl < jh) {
                                const int jm = (jl + jh + 1) >> 1;
                                if ((__float_as_int(rec[14][jm]) >> 6) <= it)
                                    jl = jm;
                                else
                                    jh = jm - 1;
                            }
                            const int e = __float_as_int(rec[14][jl]);
                            src = e & 63;
                            run = __float_as_int(rec[15][jl]) + (it - (e >> 6));
                        };
                        // one loop per specialisation keeps the two walks' registers apart
                        if (all_in) {
                            for (int it = lane; it < items; it += 64) {
                                int src, run;
                                item(it, src, run);
                                nc_fwd_item<K, true, kNCRun>(volb, colstride, P.nz, run * kNCRun,
                                                             rec, src, w, V.cu, V.cv - (float)r0,
                                                             P.eps, i_lo, i_hi, acc, SW, R);
                            }
                        } else {
                            for (int it = lane; it < items; it += 64) {
                                int src, run;
                                item(it, src, run);
                                nc_fwd_item<K, false, kNCRun>(volb, colstride, P.nz, run * kNCRun,
                                                              rec, src, w, V.cu, V.cv - (float)r0,
                                                              P.eps, i_lo, i_hi, acc, SW, R);
                            }
                        }
                    }
                }
                while (m) {
                    const int c = __ffsll((unsigned long long)m) - 1;
                    m &= m - 1ull;
                    const int s_ix = readlane_i(ix, c), s_iy = readlane_i(iy, c);
                    const float s_x = readlane_f(xc, c), s_y = readlane_f(yc, c);
                    const float s_amp = readlane_f(amp, c);
                    const float *colp = volb + ((int64_t)s_iy * P.nx + s_ix) * colstride;
                    for (int z = lane; z < P.nz; z += 64) {
                        const float val = colp[z];
                        SFVox vx;
                        sf_voxel_noncirc(V, P, s_x, s_y, fmaf((float)z, P.dz, P.z0), (float)r0, vx);
                        const int cmin = vx.o + (int)floorf(vx.t0), cmax = vx.o + (int)floorf(vx.t3);
                        const int cs = max(cmin, i_lo), ce = min(cmax, i_hi - 1);
                        const int nc = max(ce - cs + 1, 0);
                        if (nc == 0)
                            continue;
                        SFCol cc;
                        cc.o = vx.o; cc.t0 = vx.t0; cc.t1 = vx.t1; cc.t2 = vx.t2; cc.t3 = vx.t3;
                        cc.amp = s_amp;
                        float w[K];
                        sf_cell_weights<K>(cc, cs, nc, P.eps, w);
                        int *accs = acc + (cs - i_lo);
                        const float vq = val;
                        for_rows(vx.ax, R, [&](int j, float F) {
                            const float f = F * vq;
                            int *a = accs + j * SW;
#pragma unroll
                            for (int k = 0; k < K; ++k)
                                if (k < nc)
                                    atomicAdd(a + k, to_fixed(f * w[k]));
                        });
                    }
                }
            } else {   // DD (2D fan and circular cone)
                int cmin, cmax;
                dd_column_range<DET>(V, P, xc, yc, cmin, cmax);
                const int cs = max(cmin, i_lo), ce = min(cmax, i_hi - 1);
                const int nc = valid ? max(ce - cs + 1, 0) : 0;
                float fx[K], bz[K];
                dd_cell_weights<DET, K>(V, P, xc, yc, cs, nc, fx, bz);
                if constexpr (GEOM == kFan2D) {
                    if (zend - zbeg <= kLaneItems) {
                        fan2d_lane_scatter<K>(volb + ((int64_t)iy * P.nx + ix) * colstride, zbeg,
                                              zend, r0, fx, nc, acc + (cs - i_lo), SW);
                        continue;
                    }
                }
                uint64_t m = __ballot(nc > 0);
                // 3D: stage the columns' parameters (column index, strip slot, cell count, and
                // per footprint column the overlap fraction fx and the axial map scale bz) and
                // walk the columns two per wavefront in runs of 8 slices, as in the SF loop
                float (*rec)[64] = s_colrec[STAGE || STAGE_DD ? wave : 0];
                if constexpr (STAGE_DD) {
                    rec[0][lane] = __int_as_float(iy * P.nx + ix);
                    rec[1][lane] = __int_as_float(cs - i_lo);
                    rec[2][lane] = __int_as_float(nc);
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        rec[3 + k][lane] = fx[k];
                        rec[3 + K + k][lane] = bz[k];
                    }
                    if constexpr (CTP_FWD_PAIRS) {
                        if (CTP_FWD_QUADS_DD && (P.nz & 15) == 0) {
                            // four columns at a time, 16 lanes each running 16 slices
                            while (__popcll(m) >= 4) {
                                int cq[4];
#pragma unroll
                                for (int i = 0; i < 4; ++i) {
                                    cq[i] = __ffsll((unsigned long long)m) - 1;
                                    m &= m - 1ull;
                                }
                                const int src = lane < 32 ? (lane < 16 ? cq[0] : cq[1])
                                                          : (lane < 48 ? cq[2] : cq[3]);
                                const int p_nc = max(max(__float_as_int(rec[2][cq[0]]), __float_as_int(rec[2][cq[1]])),
                                                     max(__float_as_int(rec[2][cq[2]]), __float_as_int(rec[2][cq[3]])));
                                float lfx[K], lal[K], lbe[K];
#pragma unroll
                                for (int k = 0; k < K; ++k) {
                                    lfx[k] = rec[3 + k][src];
                                    const float bk = rec[3 + K + k][src];
                                    lal[k] = fmaf(bk, zb0, V.ddC - (float)r0);
                                    lbe[k] = bk * P.dz;
                                }
                                const float *colp = volb + (int64_t)__float_as_int(rec[0][src]) * colstride;
                                int *accs = acc + __float_as_int(rec[1][src]);
                                dd_fwd_run<K, 16>(colp, P.nz, lal, lbe, lfx, p_nc, accs, SW, R, lane);
                            }
                        }
                        while (__popcll(m) >= 2) {
                            const int c1 = __ffsll((unsigned long long)m) - 1;
                            m &= m - 1ull;
                            const int c2 = __ffsll((unsigned long long)m) - 1;
                            m &= m - 1ull;
                            const int src = lane < 32 ? c1 : c2;
                            const int p_nc = max(__float_as_int(rec[2][c1]), __float_as_int(rec[2][c2]));
                            float lfx[K], lal[K], lbe[K];
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                lfx[k] = rec[3 + k][src];
                                const float bk = rec[3 + K + k][src];
                                lal[k] = fmaf(bk, zb0, V.ddC - (float)r0);
                                lbe[k] = bk * P.dz;
                            }
                            const float *colp = volb + (int64_t)__float_as_int(rec[0][src]) * colstride;
                            int *accs = acc + __float_as_int(rec[1][src]);
                            dd_fwd_run<K, 8>(colp, P.nz, lal, lbe, lfx, p_nc, accs, SW, R, lane);
                        }
                    }
                }
                while (m) {
                    const int c = __ffsll((unsigned long long)m) - 1;
                    m &= m - 1ull;
                    float sfx[K], sal[K], sbe[K];
                    int s_col, s_nc, s_slot;
                    if constexpr (STAGE_DD) {
                        auto col_i = [&](int f) -> int {
                            return __builtin_amdgcn_readfirstlane(__float_as_int(rec[f][c]));
                        };
                        s_col = col_i(0);
                        s_slot = col_i(1);
                        s_nc = col_i(2);
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            sfx[k] = __int_as_float(col_i(3 + k));
                            const float bk = __int_as_float(col_i(3 + K + k));
                            sal[k] = fmaf(bk, zb0, V.ddC - (float)r0);
                            sbe[k] = bk * P.dz;
                        }
                    } else {
                        s_col = readlane_i(iy * P.nx + ix, c);
                        s_nc = readlane_i(nc, c);
                        s_slot = readlane_i(cs, c) - i_lo;
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            sfx[k] = readlane_f(fx[k], c);
                            const float bk = readlane_f(bz[k], c);
                            sal[k] = fmaf(bk, zb0, V.ddC - (float)r0);
                            sbe[k] = bk * P.dz;
                        }
                    }
                    const float *colp = volb + (int64_t)s_col * colstride;
                    int *accs = acc + s_slot;
                    if constexpr (GEOM != kFan2D && CTP_FWD_FAST) {
                        dd_fwd_run<K, 4>(colp, P.nz, sal, sbe, sfx, s_nc, accs, SW, R, lane);
                        continue;
                    }
                    for (int zb = zbeg; zb < zend; zb += 256) {
                      float vals[4];
#pragma unroll
                      for (int q = 0; q < 4; ++q) {
                          const int z = zb + lane + 64 * q;
                          vals[q] = z < zend ? colp[z] : 0.0f;
                      }
#pragma unroll
                      for (int q = 0; q < 4; ++q) {
                        const int z = zb + lane + 64 * q;
                        if (z >= zend)
                            break;
                        const float val = vals[q];
                        if constexpr (GEOM == kFan2D) {
                            int *a = accs + (z - r0) * SW;
#pragma unroll
                            for (int k = 0; k < K; ++k)
                                if (k < s_nc)
                                    atomicAdd(a + k, to_fixed(val * sfx[k]));
                        } else {
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                if (k >= s_nc)
                                    break;
                                const float zl = fmaf(sbe[k], (float)z, sal[k]);
                                const float zh = zl + sbe[k];
                                const float vk = val * sfx[k];
                                for_dd_rows(zl, zh, R, [&](int j, float wz) {
                                    atomicAdd(accs + j * SW + k, to_fixed(vk * wz));
                                });
                            }
                        }
                      }
                    }
                }
            }
        }
        __syncthreads();
    }

    // write the strip, applying the per-cell amplitude
    for (int e = threadIdx.x; e < R * STW; e += blockDim.x) {
        const int row = e / STW, k = e - row * STW;
        const int i = i_lo + k;
        if (i >= i_hi)
            continue;
        const int j = r0 + row;
        const float qinv = qscale[2 * (GEOM == kFan2D ? j : b) + 1];
        const float val = (float)acc[row * SW + k] * qinv * cell_amp<GEOM, DET, METHOD>(V, P, i, j);
        float *dst = sino + (int64_t)b * P.sino_b_stride + (int64_t)view * P.sino_view_stride +
                     (int64_t)j * P.sino_row_stride + i;
        *dst = accumulate ? *dst + val : val;
    }
}


// ---- back projection fast path (circular SF) ----------------------------------------------
//
// Along one voxel column the projected faces [p_f, q_f] of consecutive slices are ordered and,
// in the usual geometries, disjoint and narrower than a detector row.  Voxel z's SF-TT axial
// trapezoid then rises over face z, is flat up to face z+1 and falls over face z+1, and its
// gather sum_j F2_{z,j} r_j (r_j: the row's transaxially weighted sinogram value) equals
// D(z+1) - D(z) with
//   D(f) = R(q_f) - J_f,   R(t) = integral of r up to t,
//   J_f  = integral over face f of r(v) (v - p_f) / w_f,  w_f = q_f - p_f.
// A lane walks its kZChunk slices upwards, loading each detector row once (one row ahead),
// keeping the running prefix of r and evaluating D once per face.
__device__ __forceinline__ bool sf_bwd_fast_ok(float an, float bn, float af, float bf, int z0,
                                               int z1)
{
    const float m = 1e-4f;
    const float f0 = (float)z0, f1 = (float)z1;        // first and last voxel of the run
    const float d0 = an - af, db = bn - bf;
    const bool disjoint = bn > 1e-3f && bf > 1e-3f &&
                          fmaf(db, f0, d0 - bf) <= -m && fmaf(db, f1, d0 - bf) <= -m &&
                          fmaf(-db, f0, -d0 - bn) <= -m && fmaf(-db, f1, -d0 - bn) <= -m;
    const bool narrow = fabsf(fmaf(db, f0, d0)) < 1.0f - m && fabsf(fmaf(db, f1 + 1.0f, d0)) < 1.0f - m;
    return disjoint && narrow;
}

// INSIDE: every row the walk loads (floor(p_first) .. floor(q_last) + 1) lies on the detector
// and the K footprint columns cs .. cs + K - 1 exist, so rows are read at a running 32-bit
// offset (one add per row, the K columns at immediate offsets); otherwise rows are read at
// clamped, in-bounds indices (32-bit offsets within the view) and outside rows count zero.
// All NQ + 1 faces of the chunk are walked: in a partial last chunk the faces past the top
// slice follow the same lines (the callers' fast and inside tests cover all NQ + 1 faces) and
// their slices are dropped at write-out.  D is carried doubled (2D = 2R - 2J), which removes
// two multiplications per face; the accumulation takes the factor 1/2 back.
template <int K, int NQ, bool NORM, bool INSIDE>
__device__ __forceinline__ void sf_bwd_fast(const float *__restrict__ yv, int64_t row_stride,
                                            int cs, int nu, int rows, const float (&w)[K],
                                            float an, float bn, float af, float bf, int zc0,
                                            float (&acc)[NQ])
{
    const uint32_t rs = (uint32_t)row_stride;
    uint32_t cidx[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        cidx[k] = (uint32_t)min(cs + k, nu - 1);          // weights are 0 past the footprint
    auto load_row = [&](int j) -> float {
        const int jj = min(max(j, 0), rows - 1);
        const uint32_t off = (uint32_t)jj * rs;
        float r = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k)
            r = fmaf(w[k], yv[off + cidx[k]], r);
        return (j >= 0 && j < rows) ? r : 0.0f;
    };
    const float fr = (float)rows;
    const float zs = (float)zc0;
    const float an0 = fmaf(bn, zs, an), af0 = fmaf(bf, zs, af);
    const float p0 = fminf(an0, af0);
    int jc = INSIDE ? (int)floorf(p0) : (int)floorf(fminf(fmaxf(p0, -1.0f), fr));
    // INSIDE: byte offset of row jc + 1, column cs (a 32-bit offset from the view's base, the
    // K columns at immediate offsets)
    const uint32_t rsb = rs * 4u;
    uint32_t offb = ((uint32_t)(jc + 1) * rs + (uint32_t)cs) * 4u;
    auto row_at = [&](uint32_t ob) -> const float * {
        return reinterpret_cast<const float *>(reinterpret_cast<const char *>(yv) + ob);
    };
    // Row jc + 1 is fetched ahead as raw values and weighted only when the walk moves onto it,
    // so its load latency overlaps the work in between (weighting it at once would wait for
    // the load right after issuing it).
    float nraw[K];
    bool nvalid = true;
    auto fetch_next = [&]() {
        if constexpr (INSIDE) {
            const float *rp = row_at(offb);
#pragma unroll
            for (int k = 0; k < K; ++k)
                nraw[k] = rp[k];
        } else {
            const int j = jc + 1;
            const uint32_t off = (uint32_t)min(max(j, 0), rows - 1) * rs;
#pragma unroll
            for (int k = 0; k < K; ++k)
                nraw[k] = yv[off + cidx[k]];
            nvalid = j >= 0 && j < rows;
        }
    };
    auto weigh_next = [&]() -> float {
        float r = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k)
            r = fmaf(w[k], nraw[k], r);
        return nvalid ? r : 0.0f;
    };
    float rc = 0.0f;
    if constexpr (INSIDE) {
        const float *rp = row_at(offb - rsb);
#pragma unroll
        for (int k = 0; k < K; ++k)
            rc = fmaf(w[k], rp[k], rc);
    } else {
        rc = load_row(jc);
    }
    fetch_next();
    float rp = 0.0f, RP = 0.0f, D2prev = 0.0f;
    float mprev = 0.0f;                               // p + q of the previous face (NORM)
#pragma unroll
    for (int f = 0; f <= NQ; ++f) {
        const float vn = f == 0 ? an0 : fmaf((float)f, bn, an0);
        const float vf = f == 0 ? af0 : fmaf((float)f, bf, af0);
        const float p = fminf(vn, vf), q = fmaxf(vn, vf), wf = q - p;
        const int jq = INSIDE ? (int)floorf(q) : (int)floorf(fminf(fmaxf(q, -1.0f), fr));
        while (jc < jq) {
            RP += rc;
            rp = rc;
            rc = weigh_next();
            ++jc;
            if constexpr (INSIDE)
                offb += rsb;
            fetch_next();
        }
        const float fjc = (float)jc;
        // ramp-weighted integral of r over the face, doubled (branch-free: a <= 0 when the face
        // lies within row jc; a <= w keeps a^2 / w finite for a degenerate face)
        const float a = fmaxf(fjc - p, 0.0f);
        const float J2 = fmaf(rp - rc, (a * a) * fast_rcp(fmaxf(wf, 1e-30f)), rc * wf);
        const float D2 = fmaf(2.0f, fmaf(q - fjc, rc, RP), -J2);
        if (f > 0) {
            if constexpr (NORM)   // recon mode: divide by the slice's trapezoid area
                acc[f - 1] += fdiv(D2 - D2prev, (p + q) - mprev);
            else
                acc[f - 1] = fmaf(0.5f, D2 - D2prev, acc[f - 1]);
            // keep the update here: sunk to the end of the view, it would hold every face's
            // walk state live across the later faces' row loops
            asm volatile("" : "+v"(acc[f - 1]));
        }
        D2prev = D2;
        if constexpr (NORM)
            mprev = p + q;
    }
}

// Gather of one view into a lane's kZChunk voxels of a circular-scan column (SF / recon-mode
// SF): the walk when the column's faces allow it, otherwise the per-voxel fallback.
template <int K, bool NORM>
__device__ __forceinline__ void sf_circ_gather(const Params &P, const float *__restrict__ yv, int cs,
                                               int nc, const float (&w)[K], float an, float bn,
                                               float af, float bf, int zc0,
                                               float (&acc)[kZChunk])
{
    const int rows_total = P.nv, nzv = P.nz;
    const float *yc0 = yv + cs;
    if (CTP_BWD_FAST && sf_bwd_fast_ok(an, bn, af, bf, zc0, zc0 + kZChunk - 1)) {
        // rows loaded: floor(p at zc0) .. floor(q at zc0 + kZChunk) + 1
        const float z0f = (float)zc0, z1f = (float)(zc0 + kZChunk);
        const float plo = fminf(fmaf(bn, z0f, an), fmaf(bf, z0f, af));
        const float qhi = fmaxf(fmaf(bn, z1f, an), fmaf(bf, z1f, af));
        bool inside = plo >= 0.0f && qhi < (float)(rows_total - 2) && cs + K <= P.nu;
        // one walk per wavefront: when some of its lanes need the clamped walk, all take it
        // (else the wavefront would run both, one after the other)
        if (CTP_BWD_INSIDE_WAVE)
            inside = __ballot(inside) == __ballot(true);
        if (inside)
            sf_bwd_fast<K, kZChunk, NORM, true>(
                yv, P.sino_row_stride, cs, P.nu, rows_total, w, an, bn, af, bf,
                zc0, acc);
        else
            sf_bwd_fast<K, kZChunk, NORM, false>(
                yv, P.sino_row_stride, cs, P.nu, rows_total, w, an, bn, af, bf,
                zc0, acc);
        return;
    }
    // per-voxel fallback (rare: overlapping or wide faces), kept rolled so
    // that it does not set the kernel's register count
#pragma unroll 1
    for (int q = 0; q < kZChunk; ++q) {
        const int z = zc0 + q;
        if (z < nzv) {
            const Trap tr = sf_axial(an, bn, af, bf, (float)z, P.eps);
            float s = 0.0f;
            for_rows(tr, rows_total, [&](int j, float F) {
                const float *yr = yc0 + (int64_t)j * P.sino_row_stride;
                float rs = 0.0f;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (k < nc)
                        rs = fmaf(w[k], yr[k], rs);
                s = fmaf(F, rs, s);
            });
            if constexpr (NORM)
                s = fdiv(s, trap_area(tr));
#pragma unroll
            for (int qq = 0; qq < kZChunk; ++qq)
                acc[qq] += qq == q ? s : 0.0f;
        }
    }
}

// Gather of one view into a lane's kZChunk voxels of a circular-scan column (DD): the
// running-integral walk when every footprint column maps z increasingly, otherwise per voxel.
template <int K>
__device__ __forceinline__ void dd_circ_gather(const Params &P, const float *__restrict__ yv, int cs,
                                               int nc, const float (&fx)[K], const float (&al)[K],
                                               const float (&be)[K], int zc0,
                                               float (&acc)[kZChunk])
{
    const int rows_total = P.nv, nzv = P.nz;
    const float *yc0 = yv + cs;
    bool walk = true;
#pragma unroll
    for (int k = 0; k < K; ++k)
        walk = walk && !(k < nc && !(be[k] > 0.0f));
    if (CTP_BWD_FAST && walk) {
        // Footprint column k maps slice z onto rows [zeta_z, zeta_{z+1}],
        // zeta_f = al_k + be_k f, which tile the axis; the slice's gather is
        // R_k(zeta_{z+1}) - R_k(zeta_z), R_k the running integral of the column's
        // rows (clamped to the detector), so each row is loaded once.
        // all kZChunk + 1 boundaries are walked (clamped to the detector);
        // slices past the top one are dropped at write-out
        const float fr = (float)rows_total;
        const uint32_t rsb = (uint32_t)P.sino_row_stride * 4u;
        const float zc0f = (float)zc0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k >= nc)
                break;
            const float a0 = fmaf(be[k], zc0f, al[k]);
            float RP = 0.0f, Dprev = 0.0f, rc = 0.0f;
            int jc = 0;
            uint32_t offb = 0;     // byte offset of row jc, cell cs + k, in the view
            auto row_at = [&](uint32_t ob) -> float {
                return *reinterpret_cast<const float *>(
                    reinterpret_cast<const char *>(yv) + ob);
            };
#pragma unroll
            for (int f = 0; f <= kZChunk; ++f) {
                const float t = fminf(fmaxf(f == 0 ? a0 : fmaf((float)f, be[k], a0), 0.0f), fr);
                const int jt = min((int)t, rows_total - 1);
                if (f == 0) {
                    jc = jt;
                    offb = ((uint32_t)jc * (uint32_t)P.sino_row_stride +
                            (uint32_t)(cs + k)) * 4u;
                    rc = row_at(offb);
                }
                while (jc < jt) {
                    RP += rc;
                    ++jc;
                    offb += rsb;
                    rc = row_at(offb);
                }
                const float D = fmaf(t - (float)jc, rc, RP);
                if (f > 0) {
                    acc[f - 1] = fmaf(fx[k], D - Dprev, acc[f - 1]);
                    // keep the update here (see sf_bwd_fast)
                    asm volatile("" : "+v"(acc[f - 1]));
                }
                Dprev = D;
            }
        }
        return;
    }
    // per-voxel fallback, kept rolled (see sf_circ_gather)
#pragma unroll 1
    for (int q = 0; q < kZChunk; ++q) {
        const int z = zc0 + q;
        if (z < nzv) {
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k < nc) {
                    const float zl = fmaf(be[k], (float)z, al[k]);
                    const float zh = zl + be[k];
                    float rs = 0.0f;
                    for_dd_rows(zl, zh, rows_total, [&](int j, float wz) {
                        rs = fmaf(wz, yc0[(int64_t)j * P.sino_row_stride + k], rs);
                    });
                    s = fmaf(fx[k], rs, s);
                }
            }
#pragma unroll
            for (int qq = 0; qq < kZChunk; ++qq)
                acc[qq] += qq == q ? s : 0.0f;
        }
    }
}

// Back projection of one view into a lane's kZChunk voxels of a non-circular column: the walk
// of sf_bwd_fast (running integral of each detector row, one load per row) with the K + 1
// cells of the chunk carried separately, since the transaxial weights differ per voxel: voxel
// z gathers sum_k w_k(z) (D_k(z + 1) - D_k(z)).  The corners are expanded about the chunk's
// first slice and face as in the forward runs.  A face's v-interval is spanned by two corners
// (the same at both ends of the chunk: two lines) or, in the chunk where the nearest and
// farthest corners trade places, by the minimum and maximum of all four.  Returns false,
// having added nothing, when the chunk's transaxial corner order changes, its faces overlap or
// are wider than a row, or a corner's depth is not positive; the caller then takes the
// per-voxel path.
template <int K>
__device__ __forceinline__ bool nc_bwd_chunk(const ViewRec &V, const Params &P,
                                             const NCView &w, const float *__restrict__ yv,
                                             float xc, float yc, int zc0, float amp,
                                             float (&acc)[kZChunk])
{
    constexpr int NQ = kZChunk;
    const float hx = 0.5f * P.dx, hy = 0.5f * P.dy;
    const float zc = fmaf((float)zc0, P.dz, P.z0);
    const float A = fmaf(xc, V.eu[0], fmaf(yc, V.eu[1], fmaf(zc, V.eu[2], -V.seu)));
    const float W = V.sn - fmaf(xc, V.n[0], fmaf(yc, V.n[1], zc * V.n[2]));
    const float Hf = fmaf(xc, V.ev[0], fmaf(yc, V.ev[1], fmaf(zc - 0.5f * P.dz, V.ev[2], -V.sev)));
    const float Wf = W - 0.5f * w.bW;
    const float fq = (float)NQ, jl = (float)(NQ - 1);
    // transaxial corners about slice zc0 (columns), sorted by u there, with u at the last slice
    float T0[4], ts[4], tc[4], ke[4];
    // faces: the corners with the smallest / largest v at face zc0 and at face zc0 + NQ
    float NVk[4], DVk[4];
    float NVn = 0.0f, DVn = 1.0f, NVx = 0.0f, DVx = 1.0f;
    float vn0 = 3.0e38f, vx0 = -3.0e38f, vn1 = 3.0e38f, vx1 = -3.0e38f;
    int in0 = 0, ix0 = 0, in1 = 0, ix1 = 0;
    float dmin = 3.0e38f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float sx = (k & 1) ? hx : -hx, sy = (k & 2) ? hy : -hy;
        const float dW = fmaf(sx, V.n[0], sy * V.n[1]);
        const float DU = W - dW, DV = Wf - dW;
        dmin = fminf(dmin, fminf(DU, fminf(DV, fmaf(fq, w.bW, DV))));
        nc_expand(V.Du * fmaf(sx, V.eu[0], fmaf(sy, V.eu[1], A)), DU, w.aU, w.bW, T0[k], ts[k],
                  tc[k]);
        T0[k] += V.cu;
        ke[k] = fmaf(jl, fmaf(jl, tc[k], ts[k]), T0[k]);
        const float NV = V.Dv * fmaf(sx, V.ev[0], fmaf(sy, V.ev[1], Hf));
        NVk[k] = NV;
        DVk[k] = DV;
        const float a = fdiv(NV, DV), b = fdiv(fmaf(fq, w.aV, NV), fmaf(fq, w.bW, DV));
        if (a < vn0) { vn0 = a; in0 = k; NVn = NV; DVn = DV; }
        if (a > vx0) { vx0 = a; ix0 = k; NVx = NV; DVx = DV; }
        if (b < vn1) { vn1 = b; in1 = k; }
        if (b > vx1) { vx1 = b; ix1 = k; }
    }
    auto ce = [&](int i, int j) {
        const bool sw = T0[j] < T0[i];
        const float a0 = T0[i], a1 = ts[i], a2 = tc[i], a3 = ke[i];
        T0[i] = sw ? T0[j] : a0; T0[j] = sw ? a0 : T0[j];
        ts[i] = sw ? ts[j] : a1; ts[j] = sw ? a1 : ts[j];
        tc[i] = sw ? tc[j] : a2; tc[j] = sw ? a2 : tc[j];
        ke[i] = sw ? ke[j] : a3; ke[j] = sw ? a3 : ke[j];
    };
    ce(0, 1); ce(2, 3); ce(0, 2); ce(1, 3); ce(1, 2);
    // face lines: E[0] the lowest corner and E[1] the highest (two lines), or E[k] corner k
    const bool two = in0 == in1 && ix0 == ix1;
    float E0[4], Es[4], Ec[4];
    if (two) {
        nc_expand(NVn, DVn, w.aV, w.bW, E0[0], Es[0], Ec[0]);
        nc_expand(NVx, DVx, w.aV, w.bW, E0[1], Es[1], Ec[1]);
        E0[2] = E0[0], Es[2] = Es[0], Ec[2] = Ec[0];
        E0[3] = E0[1], Es[3] = Es[1], Ec[3] = Ec[1];
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            nc_expand(NVk[k], DVk[k], w.aV, w.bW, E0[k], Es[k], Ec[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        E0[k] += V.cv;
    auto ef = [&](int k, int f) {
        return f == 0 ? E0[k] : fmaf((float)f, fmaf((float)f, Ec[k], Es[k]), E0[k]);
    };
    auto pf4 = [&](int f) { return fminf(fminf(ef(0, f), ef(1, f)), fminf(ef(2, f), ef(3, f))); };
    auto qf4 = [&](int f) { return fmaxf(fmaxf(ef(0, f), ef(1, f)), fmaxf(ef(2, f), ef(3, f))); };
    // p(f + 1) - q(f) is a minimum and q(f) - p(f) a maximum of differences of corner lines
    // that are affine in f up to the expansion's remainder, so their extremes over the chunk
    // lie at its ends
    const float m = 1e-4f;
    const bool ok = dmin > 0.0f && ke[0] <= ke[1] && ke[1] <= ke[2] && ke[2] <= ke[3] &&
                    pf4(1) - qf4(0) >= m && pf4(NQ) - qf4(NQ - 1) >= m &&     // disjoint
                    qf4(0) - pf4(0) < 1.0f - m && qf4(NQ) - pf4(NQ) < 1.0f - m;  // narrow
    if (!ok)
        return false;
    // the chunk's cells c_lo .. c_lo + K (its corners drift by less than one cell)
    const float o = floorf(fminf(fmaxf(fminf(T0[0], ke[0]), -1.0e7f), 1.0e7f));
    const float hi = fminf(fmaxf(fmaxf(T0[3], ke[3]), -1.0e7f), 1.0e7f);
    const int c_lo = (int)o;
    if ((int)floorf(hi) < 0 || c_lo >= P.nu)
        return true;                       // the whole chunk projects beside the detector
#pragma unroll
    for (int k = 0; k < 4; ++k)
        T0[k] -= o;
    const int rows = P.nv;
    // the walk, once per face form (only the chosen one runs)
    auto pf2 = [&](int f) { return ef(0, f); };
    auto qf2 = [&](int f) { return ef(1, f); };
    auto walk = [&](auto pf, auto qf) -> bool {
        const float p0 = pf(0), qN = qf(NQ);
        if (qN < 0.0f || p0 >= (float)rows)
            return true;                       // the chunk's faces miss the detector rows
        const bool inside = p0 >= 0.0f && qN < (float)(rows - 2) && c_lo >= 0 &&
                            c_lo + K < P.nu;
        const uint32_t rs = (uint32_t)P.sino_row_stride;
        uint32_t cidx[K + 1];
        float cval[K + 1];                     // 1 for cells on the detector, else 0
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            const int cc = c_lo + k;
            cidx[k] = (uint32_t)min(max(cc, 0), P.nu - 1);
            cval[k] = (cc >= 0 && cc < P.nu) ? 1.0f : 0.0f;
        }
        int jc = inside ? (int)floorf(p0) : (int)floorf(fminf(fmaxf(p0, -1.0f), (float)rows));
        float nraw[K + 1], rc[K + 1], rp[K + 1], RP2[K + 1], D2p[K + 1];
        auto load_row = [&](int j, float (&dst)[K + 1]) {
            if (inside) {
                const float *rp_ = yv + (uint32_t)j * rs + (uint32_t)c_lo;
#pragma unroll
                for (int k = 0; k <= K; ++k)
                    dst[k] = rp_[k];
            } else {
                const bool jv = j >= 0 && j < rows;
                const uint32_t off = (uint32_t)min(max(j, 0), rows - 1) * rs;
#pragma unroll
                for (int k = 0; k <= K; ++k)
                    dst[k] = jv ? yv[off + cidx[k]] * cval[k] : 0.0f;
            }
        };
        load_row(jc, rc);
        load_row(jc + 1, nraw);
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            rp[k] = 0.0f;
            RP2[k] = 0.0f;
            D2p[k] = 0.0f;
        }
        const float hamp = 0.5f * amp;         // D is carried doubled
        // transaxial corners of the current voxel by second differences, with the corners' mean
        // second-order coefficient (as in the forward runs)
        const float tc2 = 0.5f * ((tc[0] + tc[1]) + (tc[2] + tc[3]));
        float tx[4], td[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            tx[k] = T0[k];
            td[k] = ts[k] + 0.5f * tc2;
        }
        const float fr = (float)rows;
#pragma unroll
        for (int f = 0; f <= NQ; ++f) {
            const float p = pf(f), q = qf(f), wf = q - p;
            const int jq = inside ? min((int)floorf(q), rows - 2)
                                  : (int)floorf(fminf(fmaxf(q, -1.0f), fr));
            while (jc < jq) {
#pragma unroll
                for (int k = 0; k <= K; ++k) {
                    RP2[k] = fmaf(2.0f, rc[k], RP2[k]);
                    rp[k] = rc[k];
                    rc[k] = nraw[k];
                }
                ++jc;
                load_row(jc + 1, nraw);
            }
            const float fjc = (float)jc;
            const float a = fmaxf(fjc - p, 0.0f);
            const float aw = (a * a) * fast_rcp(fmaxf(wf, 1e-30f));
            // 2D = 2 (R(q) - J) = 2 (qr rc + RP) - (rp - rc) aw - rc wf: one line per cell, with
            // the face's coefficients of rc and rp formed once (RP2 = 2 RP)
            const float al = fmaf(2.0f, q - fjc, aw - wf), be = -aw;
            float wv[K + 1];
            if (f > 0) {
                nc_slot_weights<K>(tx, hamp, P.eps, wv);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    tx[k] += td[k];
                    td[k] += tc2;
                }
            }
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k <= K; ++k) {
                const float D2 = fmaf(al, rc[k], fmaf(be, rp[k], RP2[k]));
                if (f > 0)
                    s = fmaf(wv[k], D2 - D2p[k], s);
                D2p[k] = D2;
            }
            if (f > 0) {
                acc[f - 1] += s;
                asm volatile("" : "+v"(acc[f - 1]));
            }
        }
        return true;
    };
    return two ? walk(pf2, qf2) : walk(pf4, qf4);
}

// ============================================================================================
// Back projector
// ============================================================================================
// Circular SF / recon-mode SF back projection is built for 8 wavefronts per SIMD (64 VGPRs; a
// few spills outside the walk): measured faster than 7 at 69 VGPRs.  DD keeps the default (its
// walk would spill).
#ifndef CTP_BWD_SF_BLOCKS
#define CTP_BWD_SF_BLOCKS 8
#endif
#ifndef CTP_BWD_NC_BLOCKS
#define CTP_BWD_NC_BLOCKS 4   // non-circular: at most 128 VGPRs (K = 4 had taken 131)
#endif
template <int GEOM, int METHOD>
constexpr int bwd_min_blocks()
{
    return GEOM == kCirc && METHOD != kDD ? CTP_BWD_SF_BLOCKS : GEOM == kNonCirc ? CTP_BWD_NC_BLOCKS : 1;
}

// Whether the back projection spreads its z-chunks over the XCDs (see bwd_kernel): SF always
// (measured 2 % faster on 256^3 x 360), DD only when the volume reaches beyond the detector
// rows (its walk runs 2 % slower spread when every chunk has work).
__host__ __device__ inline bool bwd_zspread(int nzc, int method, int row_clip)
{
    return CTP_BWD_ZSPREAD && nzc >= 8 && (method != kDD || row_clip != 0);
}
// Work-groups per XCD of the back projection (the grid is 8 times this).
__host__ __device__ inline int bwd_items_per_xcd(int nzc, int n_tiles, bool spread)
{
    return spread ? ((nzc + 7) / 8) * n_tiles : (n_tiles * nzc + 7) / 8;
}
// Whether the back projection gives each XCD a band of the tiles of every z-chunk instead:
// when the volume reaches beyond the detector rows (the chunks with work form a band, which
// whole chunks per XCD share out unevenly; curved 512x512x256 x 720: SF 30.5 -> 20.1 ms, DD
// 51.6 -> 37.6 ms).  When every chunk has work the chunk orders above are faster (256^3 x
// 360: 6.20 against 6.50 ms).
__host__ __device__ inline bool bwd_tile_bands(int row_clip)
{
    return CTP_BWD_XCDTILES && row_clip != 0;
}

template <int GEOM, int DET, int METHOD, int K>
__global__ __launch_bounds__(256, (bwd_min_blocks<GEOM, METHOD>())) void bwd_kernel(
    Params P, const ViewRec *__restrict__ views, const float *__restrict__ ys,
    float *__restrict__ vol, int accumulate)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles16_x = (P.nx + 15) >> 4;
    const int n_tiles = tiles16_x * ((P.ny + 15) >> 4);
    const int nzc = (P.nz + kZChunk - 1) / kZChunk;
    // XCD-aware order: work-group i runs on XCD i % 8 and takes (z-chunk, tile) items in
    // z-chunk-major order, so the work-groups sharing an XCD's L2 gather from the same few
    // detector rows of each view.  Spread (bwd_zspread): XCD x takes the chunks x, x + 8, ...;
    // otherwise each XCD a contiguous run of the items.  A volume taller than the detector's
    // reach has its work in a band of chunks: then each XCD takes a band of the tiles of
    // every chunk instead (bwd_tile_bands).
    const int xcd = (int)(blockIdx.x & 7), kk = (int)(blockIdx.x >> 3);
    const bool spread = bwd_zspread(nzc, METHOD, P.row_clip);
    int T, zci;
    if (bwd_tile_bands(P.row_clip)) {
        // XCD x takes the x-th eighth of the tiles (a band of tile rows) of every z-chunk,
        // chunk by chunk, so that each XCD gets an equal share of the chunks with work
        const int tb = (n_tiles + 7) >> 3;
        if (kk >= nzc * tb)
            return;
        zci = kk / tb;
        T = xcd * tb + kk % tb;
        if (T >= n_tiles)
            return;
    } else if (spread) {
        zci = xcd + 8 * (kk / n_tiles);
        T = kk % n_tiles;
        if (kk >= bwd_items_per_xcd(nzc, n_tiles, true) || zci >= nzc)
            return;
    } else {
        const int per_xcd = bwd_items_per_xcd(nzc, n_tiles, false);
        const int item = xcd * per_xcd + kk;
        if (kk >= per_xcd || item >= n_tiles * nzc)
            return;
        T = item % n_tiles;
        zci = item / n_tiles;
    }
    const int ix = (T % tiles16_x) * 16 + (wave & 1) * 8 + (lane & 7);
    const int iy = (T / tiles16_x) * 16 + (wave >> 1) * 8 + (lane >> 3);
    const int zc0 = zci * kZChunk;
    const int b = blockIdx.y;                 // batch item (3D); 0 in 2D
    const bool valid = ix < P.nx && iy < P.ny;
    const float xc = fmaf((float)ix, P.dx, P.x0), yc = fmaf((float)iy, P.dy, P.y0);
    const float hz = 0.5f * P.dz;
    const float rdiag = 0.5f * sqrtf(fmaf(P.dx, P.dx, P.dy * P.dy));   // half-diagonal (xy)
    const float *ysb = ys + (int64_t)b * P.sino_b_stride;
    const int nzv = P.nz;
    const int rows_total = GEOM == kFan2D ? P.nz : P.nv;

    float acc[kZChunk];
#pragma unroll
    for (int q = 0; q < kZChunk; ++q)
        acc[q] = 0.0f;
    if (accumulate == 2 && valid) {
        // a later launch of a view-split call: continue the sums of the earlier views
        const float *vs = vol + (GEOM == kFan2D ? 0 : (int64_t)b * P.vol_b_stride) +
                          (int64_t)iy * P.nx + ix;
#pragma unroll
        for (int q = 0; q < kZChunk; ++q)
            if (zc0 + q < nzv)
                acc[q] = vs[(int64_t)(zc0 + q) * P.vol_z_stride];
    }

    if (valid) {
        for (int view = P.v_begin; view < P.v_begin + P.v_count; ++view) {
            const ViewRec &V = views[view];
            const float *yv = ysb + (int64_t)view * P.sino_view_stride;
            const float zb0 = P.z0 - hz - V.s[2];

            if constexpr (METHOD != kDD && GEOM != kNonCirc) {
                if (GEOM != kFan2D && DET == kCurved && CTP_BWD_SKIP && CTP_BWD_PRESKIP &&
                    P.row_clip) {
                    // before the curved detector's transaxial set-up (five arc tangents): the
                    // corners' distances from the source in the transaxial plane lie within
                    // rdiag of the centre's M, so the column's axial lines v = cv + A h have
                    // slopes A in [Dv / (M + rdiag), Dv / (M - rdiag)]; when every such line
                    // misses the detector rows over the chunk's face heights h, so do the
                    // column's own (bilinear in A and h: the extremes lie at the corners).
                    // (On a flat detector the set-up is cheap and the test measured slower.)
                    const float ac = fmaf(xc, V.eu[0], fmaf(yc, V.eu[1], -V.seu));
                    const float Wc = V.sn - fmaf(xc, V.n[0], yc * V.n[1]);
                    const float M = sqrtf(fmaf(ac, ac, Wc * Wc));
                    if (M > 2.0f * rdiag) {
                        const float Ahi = fdiv(V.Dv, M - rdiag), Alo = fdiv(V.Dv, M + rdiag);
                        const float h0 = fmaf((float)zc0, P.dz, zb0);
                        const float h1 = fmaf((float)(zc0 + kZChunk), P.dz, zb0);
                        const float vlo = V.cv + fminf(fminf(Ahi * h0, Alo * h0), fminf(Ahi * h1, Alo * h1));
                        const float vhi = V.cv + fmaxf(fmaxf(Ahi * h0, Alo * h0), fmaxf(Ahi * h1, Alo * h1));
                        // a margin of 1/64 row covers the rounding of both tests
                        if (vhi < -0.015625f || vlo >= (float)rows_total + 0.015625f)
                            continue;
                    }
                }
                SFCol col;
                sf_column<DET>(V, P, xc, yc, 0.0f, col);
                if constexpr (METHOD == kSFR)
                    col.amp = sf_recon_col_amp<DET>(V, col, xc, yc);
                const int cmin = col.o + (int)floorf(col.t0), cmax = col.o + (int)floorf(col.t3);
                const int cs = max(cmin, 0), ce = min(cmax, P.nu - 1);
                const int nc = ce - cs + 1;
                if (nc <= 0)
                    continue;
                const float an = fmaf(col.An, zb0, V.cv), bn = col.An * P.dz;
                const float af = fmaf(col.Af, zb0, V.cv), bf = col.Af * P.dz;
                if (GEOM != kFan2D && CTP_BWD_SKIP && P.row_clip) {
                    // the chunk's faces (all of them lie between these lines' values at its
                    // first and last face) miss the detector rows: every row the gather would
                    // read is off the detector and adds an exact zero
                    const float z0f = (float)zc0, z1f = (float)(zc0 + kZChunk);
                    const float n0 = fmaf(bn, z0f, an), n1 = fmaf(bn, z1f, an);
                    const float f0 = fmaf(bf, z0f, af), f1 = fmaf(bf, z1f, af);
                    if (fmaxf(fmaxf(n0, n1), fmaxf(f0, f1)) < 0.0f ||
                        fminf(fminf(n0, n1), fminf(f0, f1)) >= (float)rows_total)
                        continue;
                }
                float w[K];
                sf_cell_weights<K>(col, cs, nc, P.eps, w);
                const float *yc0 = yv + cs;
                if constexpr (GEOM == kFan2D) {
#pragma unroll
                    for (int q = 0; q < kZChunk; ++q) {
                        const int z = zc0 + q;
                        if (z < nzv) {
                            const float *yr = yc0 + (int64_t)z * P.sino_row_stride;
                            float s = 0.0f;
#pragma unroll
                            for (int k = 0; k < K; ++k)
                                if (k < nc)
                                    s = fmaf(w[k], yr[k], s);
                            acc[q] += s;
                        }
                    }
                } else {
                    sf_circ_gather<K, METHOD == kSFR>(P, yv, cs, nc, w, an, bn, af, bf, zc0,
                                                     acc);
                }
            } else if constexpr (METHOD == kSF && GEOM == kNonCirc) {
                const float amp = sf_amp(V, P, xc, yc);
                if constexpr (nc_fwd_runs<GEOM, METHOD, K>()) {
                    if (P.nc_runs && nc_bwd_chunk<K>(V, P, nc_view(V, P), yv, xc, yc, zc0, amp, acc))
                        continue;
                }
                // per-voxel path, kept rolled (see sf_circ_gather)
#pragma unroll 1
                for (int q = 0; q < kZChunk; ++q) {
                    const int z = zc0 + q;
                    if (z < nzv) {
                        SFVox vx;
                        sf_voxel_noncirc(V, P, xc, yc, fmaf((float)z, P.dz, P.z0), 0.0f, vx);
                        const int cmin = vx.o + (int)floorf(vx.t0), cmax = vx.o + (int)floorf(vx.t3);
                        const int cs = max(cmin, 0), ce = min(cmax, P.nu - 1);
                        const int nc = ce - cs + 1;
                        if (nc > 0) {
                            SFCol cc;
                            cc.o = vx.o; cc.t0 = vx.t0; cc.t1 = vx.t1; cc.t2 = vx.t2; cc.t3 = vx.t3;
                            cc.amp = amp;
                            float w[K];
                            sf_cell_weights<K>(cc, cs, nc, P.eps, w);
                            float s = 0.0f;
                            for_rows(vx.ax, rows_total, [&](int j, float F) {
                                const float *yr = yv + cs + (int64_t)j * P.sino_row_stride;
                                float rs = 0.0f;
#pragma unroll
                                for (int k = 0; k < K; ++k)
                                    if (k < nc)
                                        rs = fmaf(w[k], yr[k], rs);
                                s = fmaf(F, rs, s);
                            });
#pragma unroll
                            for (int qq = 0; qq < kZChunk; ++qq)
                                acc[qq] += qq == q ? s : 0.0f;
                        }
                    }
                }
            } else {   // DD
                int cmin, cmax;
                dd_column_range<DET>(V, P, xc, yc, cmin, cmax);
                const int cs = max(cmin, 0), ce = min(cmax, P.nu - 1);
                const int nc = ce - cs + 1;
                if (nc <= 0)
                    continue;
                float fx[K], bz[K];
                dd_cell_weights<DET, K>(V, P, xc, yc, cs, nc, fx, bz);
                const float *yc0 = yv + cs;
                if constexpr (GEOM == kFan2D) {
#pragma unroll
                    for (int q = 0; q < kZChunk; ++q) {
                        const int z = zc0 + q;
                        if (z < nzv) {
                            const float *yr = yc0 + (int64_t)z * P.sino_row_stride;
                            float s = 0.0f;
#pragma unroll
                            for (int k = 0; k < K; ++k)
                                if (k < nc)
                                    s = fmaf(fx[k], yr[k], s);
                            acc[q] += s;
                        }
                    }
                } else {
                    float al[K], be[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        al[k] = fmaf(bz[k], zb0, V.ddC);
                        be[k] = bz[k] * P.dz;
                    }
                    if (CTP_BWD_SKIP && P.row_clip) {
                        // the chunk's slices map off the detector rows in every footprint
                        // column: the gather would add exact zeros
                        bool meets = false;
                        const float z0f = (float)zc0, z1f = (float)(zc0 + kZChunk);
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            const float t0 = fmaf(be[k], z0f, al[k]), t1 = fmaf(be[k], z1f, al[k]);
                            meets = meets || (k < nc && fmaxf(t0, t1) > 0.0f &&
                                              fminf(t0, t1) < (float)rows_total);
                        }
                        if (!meets)
                            continue;
                    }
                    dd_circ_gather<K>(P, yv, cs, nc, fx, al, be, zc0, acc);
                }
            }
        }
    }

    if (valid) {
        float *vb = vol + (GEOM == kFan2D ? 0 : (int64_t)b * P.vol_b_stride) +
                    (int64_t)iy * P.nx + ix;
#pragma unroll
        for (int q = 0; q < kZChunk; ++q) {
            const int z = zc0 + q;
            if (z < nzv) {
                float *dst = vb + (int64_t)z * P.vol_z_stride;
                *dst = accumulate == 1 ? *dst + acc[q] : acc[q];
            }
        }
    }
}

// ============================================================================================
// Helpers: z-fastest copy of the volume, amplitude-scaled copy of the sinogram
// ============================================================================================
// max |x| of each block of one batch item: grid (blocks per item, items); an item is the
// contiguous span of item_elems elements (a volume in 3D, an image in 2D).
template <typename T>
__global__ __launch_bounds__(256) void item_max_kernel(const T *__restrict__ in, int64_t n_items,
                                                       int64_t item_elems,
                                                       float *__restrict__ blockmax)
{
    __shared__ float wmax[4];
    for (int64_t item = blockIdx.y; item < n_items; item += gridDim.y) {
        const T *src = in + item * item_elems;
        float m = 0.0f;
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < item_elems;
             i += (int64_t)gridDim.x * 256)
            m = fmaxf(m, fabsf(to_f32(src[i])));
        for (int off = 32; off > 0; off >>= 1)
            m = fmaxf(m, __shfl_xor(m, off));
        __syncthreads();          // wmax of the previous item has been read
        if ((threadIdx.x & 63) == 0)
            wmax[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0)
            blockmax[item * gridDim.x + blockIdx.x] =
                fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    }
}

// Fixed-point scale of one item's forward accumulators (block = item): 2^S with S the largest
// integer such that max|x| * bound * 2^S <= 2^30 (bound: largest possible pre-amplitude sum per
// detector cell per unit density), qscale[2 item] = 2^S, qscale[2 item + 1] = 2^-S.  A zero or
// non-finite maximum gives S = 0.
__global__ __launch_bounds__(256) void qscale_kernel(const float *__restrict__ blockmax,
                                                     int64_t n_items, int bpi, float bound,
                                                     float *__restrict__ qscale)
{
    __shared__ float red[4];
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const float *bm = blockmax + item * bpi;
        float m = 0.0f;
        for (int i = threadIdx.x; i < bpi; i += 256)
            m = fmaxf(m, bm[i]);
        for (int off = 32; off > 0; off >>= 1)
            m = fmaxf(m, __shfl_xor(m, off));
        __syncthreads();          // red of the previous item has been read
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
            int S = 0;
            const float top = m * bound;
            if (top > 0.0f && isfinite(top)) {
                S = (int)floorf(30.0f - log2f(top));
                S = max(-126, min(S, 126));
            }
            qscale[2 * item] = ldexpf(1.0f, S);
            qscale[2 * item + 1] = ldexpf(1.0f, -S);
        }
    }
}

// z-fastest FP32 copy of the volume, each value multiplied by its item's 2^S (a power of two:
// exact).  The item is the batch index b (3D) or the "z" index itself (2D, where the batch
// takes the place of the axial dimension).
template <typename T>
__global__ __launch_bounds__(256) void transpose_zfast_kernel(const T *__restrict__ in,
                                                              float *__restrict__ out,
                                                              const float *__restrict__ qscale,
                                                              int64_t nz, int64_t plane,
                                                              int item_is_z)
{
    __shared__ float tile[32][33];
    const int64_t b = blockIdx.z;
    const int64_t p0 = (int64_t)blockIdx.x * 32, z0 = (int64_t)blockIdx.y * 32;
    const T *src = in + b * nz * plane;
    float *dst = out + b * nz * plane;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int64_t z = z0 + r, p = p0 + tx;
        if (z < nz && p < plane)
            tile[r][tx] = to_f32(src[z * plane + p]);
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t p = p0 + r, z = z0 + tx;
        if (z < nz && p < plane)
            dst[p * nz + z] = tile[tx][r] * qscale[2 * (item_is_z ? z : b)];
    }
}

// One work-group row per sinogram row (row, view, batch item), grid-strided over all rows so
// that any batch fits the grid limits.
template <int GEOM, int DET, int METHOD, typename T>
__global__ __launch_bounds__(256) void amp_scale_kernel(Params P, const ViewRec *__restrict__ views,
                                                        const T *__restrict__ in,
                                                        float *__restrict__ out, int nrows,
                                                        int64_t total_rows)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= P.nu)
        return;
    for (int64_t r = blockIdx.y; r < total_rows; r += gridDim.y) {
        const int row = (int)(r % nrows);
        const int64_t vb = r / nrows;
        const int view = (int)(vb % P.n_views);
        const int64_t b = vb / P.n_views;
        const int64_t idx = b * P.sino_b_stride + (int64_t)view * P.sino_view_stride +
                            (int64_t)row * P.sino_row_stride + i;
        out[idx] = to_f32(in[idx]) * cell_amp<GEOM, DET, METHOD>(views[view], P, i, row);
    }
}

// ---- dispatch --------------------------------------------------------------------------------

template <int GEOM, int DET, int METHOD, int K, int STW>
hipError_t fwd_launch_w(const Params &p, const ViewRec *views, const float *volT,
                        const float *qscale, float *sino, int64_t batch, int accumulate,
                        hipStream_t st)
{
    const int rows_total = GEOM == kFan2D ? p.nz : p.nv;
    const int R = min(kRowsMax, rows_total);
    size_t lds = ((size_t)(R + 1) * fwd_row_width<GEOM, METHOD, K, STW>() + kMaxCells) * sizeof(int);
    const int nchunks = (rows_total + kRowsMax - 1) / kRowsMax;
    const int n_strips = (p.nu + STW - 1) / STW;
    dim3 grid((unsigned)(CTP_FWD_XCDVIEWS ? 8 * n_strips * ((p.v_count + 7) / 8)
                                          : 8 * ((n_strips + 7) / 8) * p.v_count),
              (unsigned)((GEOM == kFan2D ? 1 : batch) * nchunks), 1);
    hipLaunchKernelGGL((fwd_kernel<GEOM, DET, METHOD, K, STW>), grid, dim3(kFwdThreads), lds, st,
                       p, views, volT, qscale, sino, accumulate, nchunks);
    return hipGetLastError();
}

template <int GEOM, int DET, int METHOD, int K>
hipError_t fwd_launch(const Params &p, const LaunchCfg &c, const ViewRec *views,
                      const float *volT, const float *qscale, float *sino, int64_t batch,
                      int accumulate, hipStream_t st)
{
    (void)c;
    // wide strips are built for the circular 3D scans with narrow footprints (the plan sets
    // strip_w accordingly)
    if constexpr (GEOM == kCirc && K <= 4) {
        if (p.strip_w == kWideStripW)
            return fwd_launch_w<GEOM, DET, METHOD, K, kWideStripW>(p, views, volT, qscale, sino,
                                                                   batch, accumulate, st);
    }
    return fwd_launch_w<GEOM, DET, METHOD, K, kStripW>(p, views, volT, qscale, sino, batch,
                                                       accumulate, st);
}

template <int GEOM, int DET, int METHOD, int K>
hipError_t bwd_launch(const Params &p, const LaunchCfg &c, const ViewRec *views,
                      const float *ysc, float *vol, int64_t batch, int accumulate,
                      hipStream_t st)
{
    (void)c;
    const int tiles = ((p.nx + 15) / 16) * ((p.ny + 15) / 16);
    const int nzc = (p.nz + kZChunk - 1) / kZChunk;
    const int per_xcd = bwd_tile_bands(p.row_clip)
                            ? nzc * ((tiles + 7) / 8)
                            : bwd_items_per_xcd(nzc, tiles, bwd_zspread(nzc, METHOD, p.row_clip));
    dim3 grid((unsigned)(8 * per_xcd), (unsigned)(GEOM == kFan2D ? 1 : batch), 1);
    hipLaunchKernelGGL((bwd_kernel<GEOM, DET, METHOD, K>), grid, dim3(256), 0, st, p, views,
                       ysc, vol, accumulate);
    return hipGetLastError();
}

template <int GEOM, int DET, int METHOD>
hipError_t amp_launch(const Params &p, const ViewRec *views, const void *in, int dtype,
                      float *out, int64_t batch, hipStream_t st)
{
    const int nrows = GEOM == kFan2D ? p.nz : p.nv;
    const int64_t total_rows = (int64_t)nrows * p.n_views * (GEOM == kFan2D ? 1 : batch);
    dim3 grid((p.nu + 255) / 256, (unsigned)std::min<int64_t>(total_rows, 65535), 1);
    if (dtype == 1)
        hipLaunchKernelGGL((amp_scale_kernel<GEOM, DET, METHOD, __hip_bfloat16>), grid, dim3(256), 0,
                           st, p, views, (const __hip_bfloat16 *)in, out, nrows, total_rows);
    else if (dtype == 2)
        hipLaunchKernelGGL((amp_scale_kernel<GEOM, DET, METHOD, __half>), grid, dim3(256), 0, st, p,
                           views, (const __half *)in, out, nrows, total_rows);
    else
        hipLaunchKernelGGL((amp_scale_kernel<GEOM, DET, METHOD, float>), grid, dim3(256), 0, st, p,
                           views, (const float *)in, out, nrows, total_rows);
    return hipGetLastError();
}

// Expand (geom, det, method, K) into a template instance.  Combinations that the plan rejects
// (non-circular + curved, non-circular + DD, recon mode off circular SF) are never
// instantiated.
template <template <int, int, int, int> class F, typename... A>
hipError_t dispatch(const LaunchCfg &c, A &&...a);

#define CTP_FOR_K(G, D, M)                                                              \
    switch (c.kcells) {                                                                 \
    case 3: return F<G, D, M, 3>::run(a...);                                            \
    case 4: return F<G, D, M, 4>::run(a...);                                            \
    case 8: return F<G, D, M, 8>::run(a...);                                            \
    default: return F<G, D, M, 16>::run(a...);                                          \
    }

template <template <int, int, int, int> class F, typename... A>
hipError_t dispatch(const LaunchCfg &c, A &&...a)
{
    if (c.geom == kFan2D && c.det == kFlat && c.method == kSF) { CTP_FOR_K(kFan2D, kFlat, kSF) }
    if (c.geom == kFan2D && c.det == kCurved && c.method == kSF) { CTP_FOR_K(kFan2D, kCurved, kSF) }
    if (c.geom == kFan2D && c.det == kFlat && c.method == kDD) { CTP_FOR_K(kFan2D, kFlat, kDD) }
    if (c.geom == kFan2D && c.det == kCurved && c.method == kDD) { CTP_FOR_K(kFan2D, kCurved, kDD) }
    if (c.geom == kCirc && c.det == kFlat && c.method == kSF) { CTP_FOR_K(kCirc, kFlat, kSF) }
    if (c.geom == kCirc && c.det == kCurved && c.method == kSF) { CTP_FOR_K(kCirc, kCurved, kSF) }
    if (c.geom == kCirc && c.det == kFlat && c.method == kDD) { CTP_FOR_K(kCirc, kFlat, kDD) }
    if (c.geom == kCirc && c.det == kCurved && c.method == kDD) { CTP_FOR_K(kCirc, kCurved, kDD) }
    if (c.geom == kNonCirc && c.det == kFlat && c.method == kSF) { CTP_FOR_K(kNonCirc, kFlat, kSF) }
    if (c.geom == kFan2D && c.det == kFlat && c.method == kSFR) { CTP_FOR_K(kFan2D, kFlat, kSFR) }
    if (c.geom == kFan2D && c.det == kCurved && c.method == kSFR) { CTP_FOR_K(kFan2D, kCurved, kSFR) }
    if (c.geom == kCirc && c.det == kFlat && c.method == kSFR) { CTP_FOR_K(kCirc, kFlat, kSFR) }
    if (c.geom == kCirc && c.det == kCurved && c.method == kSFR) { CTP_FOR_K(kCirc, kCurved, kSFR) }
    return hipErrorInvalidValue;
}
#undef CTP_FOR_K

template <int G, int D, int M, int K>
struct FwdOp {
    static hipError_t run(const Params &p, const LaunchCfg &c, const ViewRec *views,
                          const float *volT, const float *qscale, float *sino, int64_t batch,
                          int accumulate, hipStream_t st)
    {
        return fwd_launch<G, D, M, K>(p, c, views, volT, qscale, sino, batch, accumulate, st);
    }
};

template <int G, int D, int M, int K>
struct BwdOp {
    static hipError_t run(const Params &p, const LaunchCfg &c, const ViewRec *views,
                          const float *ysc, float *vol, int64_t batch, int accumulate,
                          hipStream_t st)
    {
        return bwd_launch<G, D, M, K>(p, c, views, ysc, vol, batch, accumulate, st);
    }
};

template <int G, int D, int M, int K>
struct AmpOp {
    static hipError_t run(const Params &p, const ViewRec *views, const void *in, int dtype,
                          float *out, int64_t batch, hipStream_t st)
    {
        return amp_launch<G, D, M>(p, views, in, dtype, out, batch, st);
    }
};

// ============================================================================================
// Ramp filter of filtered back projection.  A work-group filters kRampRows rows of one view.
// LDS holds the scaled ramp taps h(n), n = -np .. np-1 (np = nu rounded up to 4; taps[n + np]),
// computed once per work-group, and the current cosine-weighted row (zero past nu).  Each
// thread computes 4 consecutive outputs: per step of 4 inputs it reads the 4 row values (one
// broadcast float4) and an aligned window of 8 taps (two float4) and does 16 FMAs.
// ============================================================================================
constexpr int kRampThreads = 128;
constexpr int kRampRows = 8;

template <int DET, typename TI, typename TO>
__global__ __launch_bounds__(kRampThreads) void ramp_kernel(Params P, const ViewRec *__restrict__ views,
                                                            const TI *in, TO *out, int window,
                                                            float dbeta, int two_d)
{
    extern __shared__ float4 sm4[];
    float *sm = reinterpret_cast<float *>(sm4);
    const int nu = P.nu, np = (nu + 3) & ~3;
    float *taps = sm;                    // 2 np
    float *row = sm + 2 * np;            // np
    const int rows = two_d ? P.nz : P.nv;
    const int j0 = blockIdx.x * kRampRows;
    const int view = blockIdx.y;
    const int b = blockIdx.z;            // batch item (3D)
    const ViewRec &V = views[view];
    const float sdd = V.sdd, sad = V.sad;
    const float a = DET == kFlat ? P.du : P.du / sdd;          // pitch of the ramp samples
    const float scale = DET == kFlat ? dbeta * (sdd / sad) * P.du * 0.5f : dbeta * a / (2.0f * sad);
    const float c0 = 1.0f / (9.8696044010893586f * a * a);    // 1 / (pi a)^2
    for (int t = threadIdx.x; t < 2 * np; t += blockDim.x) {
        const int n = t - np;
        const float fn = (float)n;
        float h;
        if (window == 0)
            h = n == 0 ? 0.25f / (a * a) : ((n & 1) ? -c0 / (fn * fn) : 0.0f);
        else
            h = -2.0f * c0 / (4.0f * fn * fn - 1.0f);
        if (DET == kCurved && n != 0) {
            const float g = fn * a, r = g / sinf(g);
            h *= r * r;
        }
        taps[t] = h * scale;
    }
    // (s - d).eu: column position of the source's foot on a flat detector
    const float us = -(V.dms[0] * V.eu[0] + V.dms[1] * V.eu[1] + V.dms[2] * V.eu[2]);
    for (int j = j0; j < min(j0 + kRampRows, rows); ++j) {
        const int64_t base = (int64_t)b * P.sino_b_stride + (int64_t)view * P.sino_view_stride +
                             (int64_t)j * P.sino_row_stride;
        const float vz = two_d ? 0.0f : fmaf((float)j + 0.5f, P.dv, V.ve0) - V.sd_ev;
        __syncthreads();                 // the previous row has been consumed
        for (int k = threadIdx.x; k < np; k += blockDim.x) {
            float val = 0.0f;
            if (k < nu) {
                const float u = fmaf((float)k + 0.5f, P.du, V.ue0);
                float c;
                if (DET == kFlat) {
                    const float du_ = u - us;
                    c = sdd / sqrtf(fmaf(sdd, sdd, fmaf(du_, du_, vz * vz)));
                } else {
                    c = cosf(u / sdd) * sdd / sqrtf(fmaf(sdd, sdd, vz * vz));
                }
                val = to_f32(in[base + k]) * c;
            }
            row[k] = val;
        }
        __syncthreads();                 // the whole row is read before any output is written
        for (int i0 = 4 * threadIdx.x; i0 < np; i0 += 4 * blockDim.x) {
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
            // taps[i0 - k0 + np - 4 + m] = h(i0 - k0 - 4 + m): output r, input k0 + kk uses m = r - kk + 4
            // float4 views keep the 16-byte alignment visible (i0, np, k0 are multiples of 4)
            const float4 *wb = sm4 + ((i0 + np - 4) >> 2);
            const float4 *rv = sm4 + ((2 * np) >> 2);
#pragma unroll 4
            for (int k4 = 0; k4 < (np >> 2); ++k4) {
                const float4 x = rv[k4];
                const float4 e0 = wb[-k4];
                const float4 e1 = wb[1 - k4];
                // e0.x is not needed; keeping it live makes the compiler read whole 16-byte
                // vectors (lanes are 16 bytes apart: 32-bit reads would conflict 8-way)
                asm volatile("" : : "v"(e0.x));
                // e0 = (m0, m1, m2, m3), e1 = (m4, m5, m6, m7)
                s0 = fmaf(e1.x, x.x, s0); s0 = fmaf(e0.w, x.y, s0); s0 = fmaf(e0.z, x.z, s0); s0 = fmaf(e0.y, x.w, s0);
                s1 = fmaf(e1.y, x.x, s1); s1 = fmaf(e1.x, x.y, s1); s1 = fmaf(e0.w, x.z, s1); s1 = fmaf(e0.z, x.w, s1);
                s2 = fmaf(e1.z, x.x, s2); s2 = fmaf(e1.y, x.y, s2); s2 = fmaf(e1.x, x.z, s2); s2 = fmaf(e0.w, x.w, s2);
                s3 = fmaf(e1.w, x.x, s3); s3 = fmaf(e1.z, x.y, s3); s3 = fmaf(e1.y, x.z, s3); s3 = fmaf(e1.x, x.w, s3);
            }
            const float sv[4] = {s0, s1, s2, s3};
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (i0 + r < nu)
                    out[base + i0 + r] = from_f32<TO>(sv[r]);
        }
    }
}

template <int DET, typename TI>
hipError_t ramp_launch_out(const Params &p, const ViewRec *views, const TI *in, void *out,
                           int out_dtype, dim3 grid, size_t lds, int window, float dbeta,
                           int two_d, hipStream_t st)
{
    if (out_dtype == 1)
        hipLaunchKernelGGL((ramp_kernel<DET, TI, __hip_bfloat16>), grid, dim3(kRampThreads), lds, st,
                           p, views, in, (__hip_bfloat16 *)out, window, dbeta, two_d);
    else if (out_dtype == 2)
        hipLaunchKernelGGL((ramp_kernel<DET, TI, __half>), grid, dim3(kRampThreads), lds, st, p,
                           views, in, (__half *)out, window, dbeta, two_d);
    else
        hipLaunchKernelGGL((ramp_kernel<DET, TI, float>), grid, dim3(kRampThreads), lds, st, p,
                           views, in, (float *)out, window, dbeta, two_d);
    return hipGetLastError();
}

template <int DET>
hipError_t ramp_launch(const Params &p, const ViewRec *views, const void *in, int in_dtype,
                       void *out, int out_dtype, dim3 grid, size_t lds, int window, float dbeta,
                       int two_d, hipStream_t st)
{
    if (in_dtype == 1)
        return ramp_launch_out<DET>(p, views, (const __hip_bfloat16 *)in, out, out_dtype, grid, lds,
                                    window, dbeta, two_d, st);
    if (in_dtype == 2)
        return ramp_launch_out<DET>(p, views, (const __half *)in, out, out_dtype, grid, lds, window,
                                    dbeta, two_d, st);
    return ramp_launch_out<DET>(p, views, (const float *)in, out, out_dtype, grid, lds, window,
                                dbeta, two_d, st);
}

// FP32 workspace -> BF16 / FP16 output (optionally accumulating into it).
template <typename T>
__global__ __launch_bounds__(256) void store_convert_kernel(const float *__restrict__ src,
                                                            T *__restrict__ dst, int64_t n,
                                                            int accumulate)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float v = src[i];
        dst[i] = from_f32<T>(accumulate ? to_f32(dst[i]) + v : v);
    }
}

}  // namespace

int item_max_blocks(int64_t item_elems)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((item_elems + 8191) / 8192, 1024));
}

hipError_t launch_item_max(const void *vol, int dtype, int64_t n_items, int64_t item_elems,
                           float *blockmax, hipStream_t st)
{
    dim3 grid((unsigned)item_max_blocks(item_elems), (unsigned)std::min<int64_t>(n_items, 65535));
    if (dtype == 1)
        hipLaunchKernelGGL(item_max_kernel<__hip_bfloat16>, grid, dim3(256), 0, st,
                           (const __hip_bfloat16 *)vol, n_items, item_elems, blockmax);
    else if (dtype == 2)
        hipLaunchKernelGGL(item_max_kernel<__half>, grid, dim3(256), 0, st, (const __half *)vol,
                           n_items, item_elems, blockmax);
    else
        hipLaunchKernelGGL(item_max_kernel<float>, grid, dim3(256), 0, st, (const float *)vol,
                           n_items, item_elems, blockmax);
    return hipGetLastError();
}

hipError_t launch_transpose_zfast(const void *vol, int dtype, float *volT, const float *qscale,
                                  int64_t batch, int64_t nz, int64_t plane, int item_is_z,
                                  hipStream_t st)
{
    dim3 grid((unsigned)((plane + 31) / 32), (unsigned)((nz + 31) / 32), (unsigned)batch);
    if (dtype == 1)
        hipLaunchKernelGGL(transpose_zfast_kernel<__hip_bfloat16>, grid, dim3(256), 0, st,
                           (const __hip_bfloat16 *)vol, volT, qscale, nz, plane, item_is_z);
    else if (dtype == 2)
        hipLaunchKernelGGL(transpose_zfast_kernel<__half>, grid, dim3(256), 0, st, (const __half *)vol,
                           volT, qscale, nz, plane, item_is_z);
    else
        hipLaunchKernelGGL(transpose_zfast_kernel<float>, grid, dim3(256), 0, st, (const float *)vol,
                           volT, qscale, nz, plane, item_is_z);
    return hipGetLastError();
}

hipError_t launch_store_convert(const float *src, void *dst, int dtype, int64_t n, int accumulate,
                                hipStream_t st)
{
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    if (dtype == 1)
        hipLaunchKernelGGL(store_convert_kernel<__hip_bfloat16>, dim3(blocks), dim3(256), 0, st, src,
                           (__hip_bfloat16 *)dst, n, accumulate);
    else if (dtype == 2)
        hipLaunchKernelGGL(store_convert_kernel<__half>, dim3(blocks), dim3(256), 0, st, src,
                           (__half *)dst, n, accumulate);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_qscale(const float *blockmax, int64_t n_items, int bpi, float bound,
                         float *qscale, hipStream_t st)
{
    hipLaunchKernelGGL(qscale_kernel, dim3((unsigned)std::min<int64_t>(n_items, 65535)), dim3(256), 0,
                       st, blockmax, n_items, bpi, bound, qscale);
    return hipGetLastError();
}

hipError_t launch_amp_scale(const Params &p, const LaunchCfg &c, const ViewRec *views,
                            const void *sino, int dtype, float *out, int64_t batch, hipStream_t st)
{
    LaunchCfg c4 = c;
    c4.kcells = 3;
    return dispatch<AmpOp>(c4, p, views, sino, dtype, out, batch, st);
}

hipError_t launch_forward(const Params &p, const LaunchCfg &c, const ViewRec *views,
                          const float *volT, const float *qscale, float *sino, int64_t batch,
                          int accumulate, hipStream_t st)
{
    return dispatch<FwdOp>(c, p, c, views, volT, qscale, sino, batch, accumulate, st);
}

hipError_t launch_ramp(const Params &p, const LaunchCfg &c, const ViewRec *views, const void *in,
                       int in_dtype, void *out, int out_dtype, int64_t batch, int window,
                       float dbeta, hipStream_t st)
{
    const int two_d = c.geom == kFan2D ? 1 : 0;
    const int rows = two_d ? p.nz : p.nv;
    dim3 grid((unsigned)((rows + kRampRows - 1) / kRampRows), (unsigned)p.n_views, (unsigned)batch);
    const size_t lds = (size_t)(3 * ((p.nu + 3) & ~3)) * sizeof(float);
    if (c.det == kCurved)
        return ramp_launch<kCurved>(p, views, in, in_dtype, out, out_dtype, grid, lds, window, dbeta,
                                    two_d, st);
    return ramp_launch<kFlat>(p, views, in, in_dtype, out, out_dtype, grid, lds, window, dbeta, two_d,
                              st);
}

hipError_t launch_backward(const Params &p, const LaunchCfg &c, const ViewRec *views,
                           const float *ysc, float *vol, int64_t batch, int accumulate,
                           hipStream_t st)
{
    return dispatch<BwdOp>(c, p, c, views, ysc, vol, batch, accumulate, st);
}

// ---- library-owned scratch of the allocation-free forward entry point ----------------------
//
// One array per device (each device that loads this code object holds its own copy until the
// process ends).  In host code `scratch` only names the symbol: its device address is looked up
// once per device with hipGetSymbolAddress and cached; kernels receive that address.  Calls
// that use it share it, so overlapping calls on one device race.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;   // device -> device address of its copy of `scratch`
}  // namespace

hipError_t static_scratch(void **ptr)
{
    *ptr = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return e != hipSuccess ? e : hipErrorInvalidSymbol;
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *ptr = it->second;
    return hipSuccess;
}

}  // namespace ctp
