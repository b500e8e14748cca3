// plan.cpp -- host side of the projector library: FP64 geometry expansion (paper, Section 2.2
// and Table 1), validation, per-view device table, workspace sizing and the C ABI declared in
// include/ctproj.h.
#include "engine.h"

#include "../../include/ctproj.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

struct ctp_plan {
    ctp_geometry_desc g;     // sizes and kinds (pointers cleared)
    ctp_method method;
    ctp_mode mode;
    int device;
    ctp::ViewRec *d_views;   // device table, n_views records
    ctp::LaunchCfg cfg;
    ctp::Params base;        // geometry part of the launch constants
};

namespace {

thread_local std::string g_last_error;

ctp_status fail(ctp_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

bool sync_debug()
{
    static const bool on = [] {
        const char *e = std::getenv("CTP_SYNC_DEBUG");
        return e && e[0] && e[0] != '0';
    }();
    return on;
}

struct Vec3 {
    double x, y, z;
};
inline Vec3 operator+(Vec3 a, Vec3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline Vec3 operator-(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline Vec3 operator*(double s, Vec3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

struct Mat3 {
    double m[3][3];
    Vec3 operator*(Vec3 v) const
    {
        return {m[0][0] * v.x + m[0][1] * v.y + m[0][2] * v.z,
                m[1][0] * v.x + m[1][1] * v.y + m[1][2] * v.z,
                m[2][0] * v.x + m[2][1] * v.y + m[2][2] * v.z};
    }
    Mat3 operator*(const Mat3 &o) const
    {
        Mat3 r{};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                r.m[i][j] = m[i][0] * o.m[0][j] + m[i][1] * o.m[1][j] + m[i][2] * o.m[2][j];
        return r;
    }
};

// One view of the scan in world coordinates with the object offset removed.
struct Frame {
    Vec3 s, d, eu, ev, n;
    double sdd, ue0, ve0;     // first column / row edges (absolute detector coordinates)
};

// Per-view parameter accessor: scalar broadcast or vector.
struct ParamView {
    const double *p;
    int32_t len;
    double at(int b) const { return p == nullptr ? 0.0 : (len == 1 ? p[0] : p[b]); }
};

ctp_status check_param(const char *name, const double *p, int32_t len, int32_t n_views)
{
    if (p == nullptr && len != 0)
        return fail(CTP_EINVAL, std::string(name) + ": NULL pointer with non-zero length");
    if (p != nullptr && len != 1 && len != n_views)
        return fail(CTP_EINVAL, std::string(name) + ": length must be 1 or n_views");
    if (p != nullptr)
        for (int32_t i = 0; i < len; ++i)
            if (!std::isfinite(p[i]))
                return fail(CTP_EINVAL, std::string(name) + ": non-finite value");
    return CTP_OK;
}

// Pose R = Rz(theta) Rx(phi) Ry(psi): psi about y first, then phi about x, then theta about z,
// each counter-clockwise (Section 2.2).
Mat3 pose(double th, double ph, double ps)
{
    const double ct = std::cos(th), st = std::sin(th);
    const double cp = std::cos(ph), sp = std::sin(ph);
    const double cs = std::cos(ps), ss = std::sin(ps);
    const Mat3 Rz{{{ct, -st, 0}, {st, ct, 0}, {0, 0, 1}}};
    const Mat3 Rx{{{1, 0, 0}, {0, cp, -sp}, {0, sp, cp}}};
    const Mat3 Ry{{{cs, 0, ss}, {0, 1, 0}, {-ss, 0, cs}}};
    return Rz * (Rx * Ry);
}

}  // namespace

namespace ctp {
ctp_status set_error(ctp_status st, const std::string &msg) { return fail(st, msg); }
void clear_error() { g_last_error.clear(); }
int plan_device(const ctp_plan *plan) { return plan->device; }
double plan_work(const ctp_plan *plan)
{
    const ctp_geometry_desc &g = plan->g;
    return (double)g.nx * g.ny * (g.kind == CTP_FAN2D ? 1 : g.nz) * g.n_views;
}
int plan_views(const ctp_plan *plan) { return plan->g.n_views; }
}  // namespace ctp

extern "C" {

const char *ctp_status_string(ctp_status s)
{
    switch (s) {
    case CTP_OK: return "ok";
    case CTP_EINVAL: return "invalid argument";
    case CTP_EUNSUPPORTED: return "unsupported";
    case CTP_ENOMEM: return "out of memory";
    case CTP_EDEVICE: return "device error";
    case CTP_ETIMEOUT: return "timed out";
    case CTP_ECANCELED: return "cancelled";
    }
    return "unknown status";
}

const char *ctp_last_error(void) { return g_last_error.c_str(); }

ctp_status ctp_plan_create(const ctp_geometry_desc *desc, ctp_method method, ctp_mode mode,
                           ctp_plan **out)
{
    g_last_error.clear();
    if (desc == nullptr || out == nullptr)
        return fail(CTP_EINVAL, "NULL descriptor or output pointer");
    *out = nullptr;
    const ctp_geometry_desc &g = *desc;
    if (g.kind < CTP_FAN2D || g.kind > CTP_CONE_NONCIRC)
        return fail(CTP_EINVAL, "unknown geometry kind");
    if (g.det != CTP_DET_FLAT && g.det != CTP_DET_CURVED)
        return fail(CTP_EINVAL, "unknown detector model");
    if (method != CTP_SF && method != CTP_DD)
        return fail(CTP_EINVAL, "unknown projector method");
    if (mode != CTP_MODE_PROJ && mode != CTP_MODE_RECON)
        return fail(CTP_EINVAL, "unknown projection mode");
    const bool recon = mode == CTP_MODE_RECON;
    const bool two_d = g.kind == CTP_FAN2D;
    if (g.nx <= 0 || g.ny <= 0 || g.nu <= 0 || g.n_views <= 0 || (!two_d && (g.nz <= 0 || g.nv <= 0)))
        return fail(CTP_EINVAL, "sizes must be positive");
    if (two_d && (g.nz != 1 || g.nv != 1))
        return fail(CTP_EINVAL, "2D fan beam requires nz = nv = 1");
    if (!(g.dx > 0) || !(g.dy > 0) || !(g.du > 0) || (!two_d && (!(g.dz > 0) || !(g.dv > 0))))
        return fail(CTP_EINVAL, "spacings must be positive");
    if ((int64_t)g.nx * g.ny > (int64_t)1 << 28 || (int64_t)g.nx * g.ny * g.nz > (int64_t)1 << 34)
        return fail(CTP_EINVAL, "volume too large");
    if (g.kind == CTP_CONE_NONCIRC && g.det == CTP_DET_CURVED)
        return fail(CTP_EUNSUPPORTED, "non-circular scans use flat detectors only");
    if (method == CTP_DD && g.kind == CTP_CONE_NONCIRC)
        return fail(CTP_EUNSUPPORTED, "distance driven is built for circular scans only");
    if (recon && (method != CTP_SF || g.kind == CTP_CONE_NONCIRC))
        return fail(CTP_EUNSUPPORTED, "recon mode is built for SF on circular scans");

    struct {
        const char *name;
        const double *p;
        int32_t len;
    } prm[] = {{"theta", g.theta, g.len_theta}, {"phi", g.phi, g.len_phi}, {"psi", g.psi, g.len_psi},
               {"sad", g.sad, g.len_sad}, {"sdd", g.sdd, g.len_sdd}, {"x_src", g.x_src, g.len_x_src},
               {"z_src", g.z_src, g.len_z_src}, {"x_ofst", g.x_ofst, g.len_x_ofst},
               {"y_ofst", g.y_ofst, g.len_y_ofst}, {"z_ofst", g.z_ofst, g.len_z_ofst},
               {"u_ofst", g.u_ofst, g.len_u_ofst}, {"v_ofst", g.v_ofst, g.len_v_ofst}};
    for (auto &q : prm) {
        ctp_status st = check_param(q.name, q.p, q.len, g.n_views);
        if (st != CTP_OK)
            return st;
    }
    const ParamView theta{g.theta, g.len_theta}, phi{g.phi, g.len_phi}, psi{g.psi, g.len_psi},
        sad{g.sad, g.len_sad}, sdd{g.sdd, g.len_sdd}, xsrc{g.x_src, g.len_x_src},
        zsrc{g.z_src, g.len_z_src}, xo{g.x_ofst, g.len_x_ofst}, yo{g.y_ofst, g.len_y_ofst},
        zo{g.z_ofst, g.len_z_ofst}, uo{g.u_ofst, g.len_u_ofst}, vo{g.v_ofst, g.len_v_ofst};

    const int nz = two_d ? 1 : g.nz, nv = two_d ? 1 : g.nv;
    const double hx = 0.5 * g.nx * g.dx, hy = 0.5 * g.ny * g.dy, hz = two_d ? 0.0 : 0.5 * nz * g.dz;
    std::vector<ctp::ViewRec> recs((size_t)g.n_views);
    double kmax = 0.0;   // widest transaxial footprint (columns) over all views
    // non-circular SF column runs: remainder of the second-order expansion of a corner's
    // projection over a run, and how far a footprint drifts along a run (columns)
    double nc_rem = 0.0, nc_drift = 0.0;
    double rmax = 0.0;   // recon mode: largest SAD / W over views and volume corners
    bool row_clip = false;  // a volume corner projects beyond the detector rows in some view
    double mmin = 1e300; // smallest magnification over views and volume corners

    for (int b = 0; b < g.n_views; ++b) {
        const double ph = g.kind == CTP_CONE_NONCIRC ? phi.at(b) : 0.0;
        const double ps = g.kind == CTP_CONE_NONCIRC ? psi.at(b) : 0.0;
        if (g.kind != CTP_CONE_NONCIRC && (phi.at(b) != 0.0 || psi.at(b) != 0.0))
            return fail(CTP_EINVAL, "phi and psi must be zero for circular and 2D scans");
        if (!(sad.at(b) > 0) || !(sdd.at(b) > 0))
            return fail(CTP_EINVAL, "SAD and SDD must be positive");
        if (g.det == CTP_DET_CURVED && xsrc.at(b) != 0.0)
            return fail(CTP_EUNSUPPORTED, "curved detector with a lateral source offset");
        const Mat3 R = pose(theta.at(b), ph, ps);
        const Vec3 obj{xo.at(b), yo.at(b), two_d ? 0.0 : zo.at(b)};
        Frame f;
        f.s = R * Vec3{xsrc.at(b), sad.at(b), two_d ? 0.0 : zsrc.at(b)} - obj;
        f.d = R * Vec3{0.0, sad.at(b) - sdd.at(b), 0.0} - obj;
        f.eu = R * Vec3{1, 0, 0};
        f.ev = R * Vec3{0, 0, 1};
        f.n = R * Vec3{0, 1, 0};
        f.sdd = sdd.at(b);
        f.ue0 = -0.5 * g.nu * g.du - uo.at(b);
        f.ve0 = two_d ? -0.5 * g.dv : -0.5 * nv * g.dv - vo.at(b);

        // every corner of the volume box must lie strictly in front of the source
        double Wmin = 1e300, Wmax = 0.0, amax = 0.0, vmax = 0.0;
        for (int c = 0; c < 8; ++c) {
            const Vec3 p{(c & 1) ? hx : -hx, (c & 2) ? hy : -hy, (c & 4) ? hz : -hz};
            const double W = dot(f.s - p, f.n);
            Wmin = std::fmin(Wmin, W);
            Wmax = std::fmax(Wmax, W);
            amax = std::fmax(amax, std::fabs(dot(p - f.s, f.eu)));
            vmax = std::fmax(vmax, std::fabs(dot(p - f.s, f.ev)));
        }
        const double D = dot(f.s - f.d, f.n);
        if (!(Wmin > 1e-6 * f.sdd))
            return fail(CTP_EINVAL, "part of the volume is at or behind the source in view " + std::to_string(b));
        rmax = std::fmax(rmax, sad.at(b) / Wmin);
        if (!two_d) {
            for (int c = 0; c < 8; ++c) {
                const Vec3 p{(c & 1) ? hx : -hx, (c & 2) ? hy : -hy, (c & 4) ? hz : -hz};
                const double W = dot(f.s - p, f.n), h = dot(p - f.s, f.ev);
                const double a = dot(p - f.s, f.eu);
                const double v = dot(f.s - f.d, f.ev) +
                                 (g.det == CTP_DET_FLAT ? dot(f.s - f.d, f.n) * h / W
                                                        : f.sdd * h / std::hypot(a, W));
                const double row = (v - f.ve0) / g.dv;
                row_clip = row_clip || row < 0.0 || row > (double)nv;
            }
        }
        mmin = std::fmin(mmin, (g.det == CTP_DET_FLAT ? D : f.sdd) / std::hypot(Wmax, amax));

        // bound on the transaxial footprint width (columns): |grad u| * voxel extent
        const double grad = g.det == CTP_DET_FLAT ? D * (Wmin + amax) / (Wmin * Wmin) / g.du
                                                  : f.sdd / Wmin / g.du;
        const double ext = method == CTP_SF ? std::sqrt(g.dx * g.dx + g.dy * g.dy) : std::fmax(g.dx, g.dy);
        kmax = std::fmax(kmax, grad * ext);
        if (g.kind == CTP_CONE_NONCIRC && Wmin > 0.0) {
            // along a column a corner projects to f(j) = f0 + s j / (1 + r j) (j: slices from
            // a run's start) with r = dz n_z / W and |s| at most as below; the kernels use
            // f0 + s j + c j^2 (c = -s r), off by |s| r^2 j^3; the transaxial corners share
            // the mean of their four c, which lie within 2 |dW| / W of it (dW: a corner's depth
            // offset from the column centre)
            const double Du = (g.det == CTP_DET_FLAT ? D : f.sdd) / g.du;
            const double Dv = (g.det == CTP_DET_FLAT ? D : f.sdd) / g.dv;
            const double r = g.dz * std::fabs(f.n.z) / Wmin;
            const double su = Du * g.dz * (std::fabs(f.eu.z) + amax / Wmin * std::fabs(f.n.z)) / Wmin;
            const double sv = Dv * g.dz * (std::fabs(f.ev.z) + vmax / Wmin * std::fabs(f.n.z)) / Wmin;
            const double j = ctp::kNCRunMax;
            const double dwr = std::hypot(g.dx, g.dy) / Wmin;
            nc_rem = std::fmax(nc_rem, std::fmax(su * (r * j + dwr), sv * r * j) * r * j * j);
            nc_drift = std::fmax(nc_drift, su * (j - 1.0));
        }

        ctp::ViewRec &r = recs[(size_t)b];
        std::memset(&r, 0, sizeof(r));
        const Vec3 dms = f.d - f.s;
        const double vals_eu[3] = {f.eu.x, f.eu.y, f.eu.z}, vals_ev[3] = {f.ev.x, f.ev.y, f.ev.z};
        const double vals_n[3] = {f.n.x, f.n.y, f.n.z}, vals_s[3] = {f.s.x, f.s.y, f.s.z};
        const double vals_d[3] = {dms.x, dms.y, dms.z};
        for (int k = 0; k < 3; ++k) {
            r.eu[k] = (float)vals_eu[k];
            r.ev[k] = (float)vals_ev[k];
            r.n[k] = (float)vals_n[k];
            r.s[k] = (float)vals_s[k];
            r.dms[k] = (float)vals_d[k];
        }
        r.seu = (float)dot(f.s, f.eu);
        r.sev = (float)dot(f.s, f.ev);
        r.sn = (float)dot(f.s, f.n);
        const Vec3 smd = f.s - f.d;
        if (g.det == CTP_DET_FLAT) {
            r.Du = (float)(D / g.du);
            r.Dv = (float)(D / g.dv);
            r.cu = (float)((dot(smd, f.eu) - f.ue0) / g.du);
        } else {
            r.Du = (float)(f.sdd / g.du);
            r.Dv = (float)(f.sdd / g.dv);
            r.cu = (float)(-f.ue0 / g.du);
        }
        r.cv = (float)((dot(smd, f.ev) - f.ve0) / g.dv);
        r.ue0 = (float)f.ue0;
        r.ve0 = (float)f.ve0;
        r.sdd = (float)f.sdd;
        r.sd_ev = (float)dot(smd, f.ev);
        // distance driven: planes y = const when the detector normal is closer to y
        r.ydrv = std::fabs(f.n.y) >= std::fabs(f.n.x) ? 1 : 0;
        r.ddC = (float)(-(dms.z + f.ve0) / g.dv);
        r.sad = (float)sad.at(b);
        if (method == CTP_DD) {
            // every column-edge ray must cross the driving planes
            for (int i = 0; i <= g.nu; i += (g.nu > 1 ? g.nu : 1)) {
                const double u = f.ue0 + i * g.du;
                Vec3 q;
                if (g.det == CTP_DET_FLAT)
                    q = dms + u * f.eu;
                else
                    q = f.sdd * std::sin(u / f.sdd) * f.eu - f.sdd * std::cos(u / f.sdd) * f.n;
                const double qa = r.ydrv ? q.y : q.x;
                const double na = r.ydrv ? -f.n.y : -f.n.x;   // central ray direction component
                if (!(qa * na > 1e-3 * std::fabs(na) * std::sqrt(q.x * q.x + q.y * q.y)))
                    return fail(CTP_EINVAL, "detector ray parallel to the driving planes in view " + std::to_string(b));
            }
        }
    }
    const int need = (int)std::floor(kmax * 1.001 + 1e-6) + 2;
    if (need > ctp::kMaxCells)
        return fail(CTP_EUNSUPPORTED, "footprint wider than 16 detector columns");

    ctp_plan *plan = new (std::nothrow) ctp_plan;
    if (!plan)
        return fail(CTP_ENOMEM, "host allocation failed");
    std::memset(plan, 0, sizeof(*plan));
    plan->g = g;
    plan->method = method;
    plan->mode = mode;
    hipError_t e = hipGetDevice(&plan->device);
    if (e != hipSuccess) {
        delete plan;
        return fail(CTP_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    e = hipMalloc(&plan->d_views, recs.size() * sizeof(ctp::ViewRec));
    if (e != hipSuccess) {
        delete plan;
        return fail(e == hipErrorOutOfMemory ? CTP_ENOMEM : CTP_EDEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    e = hipMemcpy(plan->d_views, recs.data(), recs.size() * sizeof(ctp::ViewRec), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(plan->d_views);
        delete plan;
        return fail(CTP_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }

    ctp::LaunchCfg &c = plan->cfg;
    c.geom = g.kind;
    c.det = g.det;
    c.method = recon ? ctp::kSFR : method;
    c.kcells = need <= 3 ? 3 : need <= 4 ? 4 : need <= 8 ? 8 : 16;
    // Forward strips: on a short detector the strip's LDS rows are few, and wider strips share
    // each voxel column's set-up and the tile culling over more cells (512x512x256 x 720 views
    // on 64 rows, SF forward: 26.1 ms with 16 columns, 23.2 with 32, 22.5 with 64); on tall
    // detectors 16 columns keep more work-groups per CU (256^3 x 360 on 384 rows: 5.33 ms
    // against 5.84 at 32)
    const int strip_w = g.kind == CTP_CONE_CIRC && nv <= ctp::kWideStripRows && c.kcells <= 4
                            ? ctp::kWideStripW
                            : ctp::kStripW;
    c.n_strips = (g.nu + strip_w - 1) / strip_w;
    c.n_row_chunks = (nv + ctp::kRowsMax - 1) / ctp::kRowsMax;
    // Largest possible pre-amplitude sum of one detector cell per unit |x|: SF sums
    // footprint x amplitude, at most a few times the path through the volume box; DD sums
    // overlap fractions, at most one per driving plane.  Generous factors keep the forward
    // projector's fixed-point accumulators far from overflow.
    {
        const double lx = g.nx * g.dx, ly = g.ny * g.dy, lz = two_d ? 0.0 : nz * g.dz;
        c.acc_bound = method == CTP_SF ? (float)(4.0 * std::sqrt(lx * lx + ly * ly + lz * lz))
                                       : (float)(2.0 * (std::max(g.nx, g.ny) + 2));
        if (recon) {
            // normalised footprints: per layer of voxels across a ray the weights of one cell
            // sum to at most 2 max(1, cell / voxel shadow) per axis; (nx + ny + 2) layers
            const double fu = 2.0 * (1.0 + g.du / (mmin * std::min(g.dx, g.dy)));
            const double fv = two_d ? 1.0 : 2.0 * (1.0 + g.dv / (mmin * g.dz));
            c.acc_bound = (float)(2.0 * rmax * rmax * (g.nx + g.ny + 2) * fu * fv);
        }
    }

    ctp::Params &p = plan->base;
    p.nx = g.nx;
    p.ny = g.ny;
    p.nz = nz;
    p.dx = (float)g.dx;
    p.dy = (float)g.dy;
    p.dz = (float)(two_d ? 1.0 : g.dz);
    p.x0 = (float)(-0.5 * (g.nx - 1) * g.dx);
    p.y0 = (float)(-0.5 * (g.ny - 1) * g.dy);
    p.z0 = (float)(two_d ? 0.0 : -0.5 * (nz - 1) * g.dz);
    p.nu = g.nu;
    p.nv = nv;
    p.du = (float)g.du;
    p.dv = (float)(two_d ? 1.0 : g.dv);
    p.n_views = g.n_views;
    p.v_begin = 0;
    p.v_count = g.n_views;
    p.row_clip = row_clip ? 1 : 0;
    p.strip_w = strip_w;
    p.eps = 1e-6f;
    // non-circular SF column runs: expansion accurate to 2e-5 cells / rows, a run's footprints
    // within K + 1 cells (their union is narrower than K: widths below K - 1 plus the drift)
    // and the drift below one cell
    p.nc_runs = (g.kind == CTP_CONE_NONCIRC && method == CTP_SF && !recon && c.kcells <= 4 &&
                 nc_rem < 2e-5 && nc_drift < 0.999 && (kmax + nc_drift) * 1.001 < c.kcells)
                    ? 1 : 0;
    plan->g.theta = plan->g.phi = plan->g.psi = plan->g.sad = plan->g.sdd = nullptr;
    plan->g.x_src = plan->g.z_src = plan->g.x_ofst = plan->g.y_ofst = plan->g.z_ofst = nullptr;
    plan->g.u_ofst = plan->g.v_ofst = nullptr;
    *out = plan;
    return CTP_OK;
}

ctp_status ctp_plan_destroy(ctp_plan *plan)
{
    g_last_error.clear();
    if (plan == nullptr)
        return CTP_OK;
    hipError_t e = hipFree(plan->d_views);
    delete plan;
    if (e != hipSuccess)
        return fail(CTP_EDEVICE, std::string("hipFree: ") + hipGetErrorString(e));
    return CTP_OK;
}

ctp_status ctp_plan_bytes(const ctp_plan *plan, ctp_dtype dtype, int64_t batch, size_t *vol_bytes,
                          size_t *sino_bytes)
{
    g_last_error.clear();
    if (plan == nullptr || batch < 1)
        return fail(CTP_EINVAL, "NULL plan or batch < 1");
    if (dtype != CTP_F32 && dtype != CTP_BF16 && dtype != CTP_F16)
        return fail(CTP_EINVAL, "unknown dtype");
    const size_t es = dtype == CTP_F32 ? 4 : 2;
    const ctp_geometry_desc &g = plan->g;
    const bool two_d = g.kind == CTP_FAN2D;
    const size_t nvox = (size_t)g.nx * g.ny * (two_d ? 1 : g.nz);
    const size_t ncell = (size_t)g.n_views * g.nu * (two_d ? 1 : g.nv);
    if (vol_bytes)
        *vol_bytes = nvox * (size_t)batch * es;
    if (sino_bytes)
        *sino_bytes = ncell * (size_t)batch * es;
    return CTP_OK;
}

namespace {

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Forward workspace: the per-item fixed-point scales (two floats per batch item), the per-block
// max |x| of each item, the z-fastest scaled FP32 copy of the volume, then (half-precision
// sinograms only) an FP32 sinogram.
// Backward workspace: the amplitude-scaled FP32 sinogram (omitted for 2D SF with an FP32
// sinogram), then (half-precision volumes only) an FP32 volume.
struct FwdWs {
    size_t blockmax_off, volT_off, sino_off, total;
    int64_t item_elems, tr_batch, tr_nz, plane;
    int bpi;
};
struct BwdWs {
    size_t ysc_off, vol_off, total;
    bool scaled;
};

FwdWs fwd_ws_layout(const ctp_plan *plan, int64_t batch, ctp_dtype sino_dtype)
{
    const ctp_geometry_desc &g = plan->g;
    const bool two_d = g.kind == CTP_FAN2D;
    FwdWs w;
    w.plane = (int64_t)g.nx * g.ny;
    w.tr_batch = two_d ? 1 : batch;
    w.tr_nz = two_d ? batch : g.nz;
    w.item_elems = two_d ? w.plane : w.plane * g.nz;
    w.bpi = ctp::item_max_blocks(w.item_elems);
    w.blockmax_off = align256((size_t)batch * 2 * sizeof(float));
    w.volT_off = w.blockmax_off + align256((size_t)batch * w.bpi * sizeof(float));
    w.sino_off = w.volT_off + align256((size_t)w.tr_batch * w.tr_nz * w.plane * sizeof(float));
    size_t sb = 0;
    ctp_plan_bytes(plan, CTP_F32, batch, nullptr, &sb);
    w.total = w.sino_off + (sino_dtype == CTP_F32 ? 0 : sb);
    return w;
}

BwdWs bwd_ws_layout(const ctp_plan *plan, int64_t batch, ctp_dtype vol_dtype, ctp_dtype sino_dtype)
{
    size_t vb = 0, sb = 0;
    ctp_plan_bytes(plan, CTP_F32, batch, &vb, &sb);
    BwdWs w;
    // the per-cell amplitude is 1 for 2D SF and in recon mode: FP32 sinograms are read as given
    w.scaled = !(sino_dtype == CTP_F32 && (plan->mode == CTP_MODE_RECON ||
                                           (plan->g.kind == CTP_FAN2D && plan->method == CTP_SF)));
    w.ysc_off = 0;
    w.vol_off = w.scaled ? align256(sb) : 0;
    w.total = w.vol_off + (vol_dtype == CTP_F32 ? 0 : vb);
    return w;
}

}  // namespace

ctp_status ctp_workspace_bytes(const ctp_plan *plan, ctp_direction dir, ctp_dtype vol_dtype,
                               ctp_dtype sino_dtype, int64_t batch, size_t *bytes)
{
    ctp_status st = ctp_plan_bytes(plan, vol_dtype, batch, nullptr, nullptr);
    if (st == CTP_OK)
        st = ctp_plan_bytes(plan, sino_dtype, batch, nullptr, nullptr);
    if (st != CTP_OK)
        return st;
    if (bytes == nullptr)
        return fail(CTP_EINVAL, "NULL output");
    if (dir == CTP_FORWARD)
        *bytes = fwd_ws_layout(plan, batch, sino_dtype).total;
    else if (dir == CTP_BACKWARD)
        *bytes = bwd_ws_layout(plan, batch, vol_dtype, sino_dtype).total;
    else
        return fail(CTP_EINVAL, "unknown direction");
    return CTP_OK;
}

namespace {

ctp_status prepare_call(const ctp_plan *plan, const void *a, const void *b, ctp_dtype da, ctp_dtype db,
                        int64_t batch, void *ws, size_t ws_bytes, ctp_direction dir, ctp::Params &p)
{
    if (plan == nullptr || a == nullptr || b == nullptr)
        return fail(CTP_EINVAL, "NULL plan or data pointer");
    if (batch < 1)
        return fail(CTP_EINVAL, "batch must be >= 1");
    for (ctp_dtype d : {da, db})
        if (d != CTP_F32 && d != CTP_BF16 && d != CTP_F16)
            return fail(CTP_EINVAL, "unknown dtype");
    const bool two_d = plan->g.kind == CTP_FAN2D;
    if (two_d && batch > (int64_t)1 << 20)
        return fail(CTP_EINVAL, "2D batch too large (at most 2^20 images)");
    if (!two_d && batch * plan->cfg.n_row_chunks > 65535)
        return fail(CTP_EINVAL, "batch too large");
    size_t need = 0;
    const ctp_dtype vol_dt = dir == CTP_FORWARD ? da : db, sino_dt = dir == CTP_FORWARD ? db : da;
    ctp_status st = ctp_workspace_bytes(plan, dir, vol_dt, sino_dt, batch, &need);
    if (st != CTP_OK)
        return st;
    if (need > 0 && (ws == nullptr || ws_bytes < need))
        return fail(CTP_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    if (need > 0 && ((uintptr_t)ws & 255u) != 0)
        return fail(CTP_EINVAL, "workspace must be 256-byte aligned");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
        return fail(CTP_EINVAL, "plan was created on another device");
    p = plan->base;
    const ctp_geometry_desc &g = plan->g;
    const int64_t plane = (int64_t)g.nx * g.ny;
    if (two_d) {
        // the batch runs along the axial dimension: one "slice" / "row" per item
        p.nz = (int)batch;
        p.nv = (int)batch;
        p.vol_z_stride = plane;
        p.vol_b_stride = 0;
        p.sino_row_stride = (int64_t)g.n_views * g.nu;
        p.sino_view_stride = g.nu;
        p.sino_b_stride = 0;
    } else {
        p.vol_z_stride = plane;
        p.vol_b_stride = plane * g.nz;
        p.sino_row_stride = g.nu;
        p.sino_view_stride = (int64_t)g.nv * g.nu;
        p.sino_b_stride = (int64_t)g.n_views * g.nv * g.nu;
    }
    return CTP_OK;
}

ctp_status finish(hipError_t e, hipStream_t stream, const char *what)
{
    if (e == hipSuccess && sync_debug())
        e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
        return fail(CTP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return CTP_OK;
}

}  // namespace

}  // extern "C"

namespace {

// The forward projection into a validated workspace (prepare_call has run).
ctp_status project_into(const ctp_plan *plan, const void *vol, ctp_dtype vol_dtype, void *sino,
                        ctp_dtype sino_dtype, int64_t batch, int accumulate, void *workspace,
                        ctp::Params p, hipStream_t stream, int views_per_launch = 0)
{
    const FwdWs w = fwd_ws_layout(plan, batch, sino_dtype);
    char *ws = static_cast<char *>(workspace);
    float *qscale = reinterpret_cast<float *>(ws);
    float *blockmax = reinterpret_cast<float *>(ws + w.blockmax_off);
    float *volT = reinterpret_cast<float *>(ws + w.volT_off);
    const bool half_out = sino_dtype != CTP_F32;
    float *out = half_out ? reinterpret_cast<float *>(ws + w.sino_off) : static_cast<float *>(sino);
    hipError_t e = ctp::launch_item_max(vol, (int)vol_dtype, batch, w.item_elems, blockmax, stream);
    if (e == hipSuccess)
        e = ctp::launch_qscale(blockmax, batch, w.bpi, plan->cfg.acc_bound, qscale, stream);
    if (e == hipSuccess)
        e = ctp::launch_transpose_zfast(vol, (int)vol_dtype, volT, qscale, w.tr_batch, w.tr_nz,
                                        w.plane, plan->g.kind == CTP_FAN2D ? 1 : 0, stream);
    // each view's cells are written by its own work-groups, so launches over consecutive view
    // ranges give the bits of one launch over all views
    const int nv = plan->g.n_views;
    const int step = views_per_launch > 0 ? std::min(views_per_launch, nv) : nv;
    for (int v0 = 0; v0 < nv && e == hipSuccess; v0 += step) {
        p.v_begin = v0;
        p.v_count = std::min(step, nv - v0);
        e = ctp::launch_forward(p, plan->cfg, plan->d_views, volT, qscale, out, batch,
                                half_out ? 0 : accumulate, stream);
    }
    if (e == hipSuccess && half_out) {
        size_t sb = 0;
        ctp_plan_bytes(plan, CTP_F32, batch, nullptr, &sb);
        e = ctp::launch_store_convert(out, sino, (int)sino_dtype, (int64_t)(sb / 4), accumulate, stream);
    }
    return finish(e, stream, "forward projection");
}

}  // namespace

extern "C" {

ctp_status ctp_project(const ctp_plan *plan, const void *vol, ctp_dtype vol_dtype, void *sino,
                       ctp_dtype sino_dtype, int64_t batch, int accumulate, void *workspace,
                       size_t workspace_bytes, hipStream_t stream)
{
    g_last_error.clear();
    ctp::Params p;
    ctp_status st = prepare_call(plan, vol, sino, vol_dtype, sino_dtype, batch, workspace,
                                 workspace_bytes, CTP_FORWARD, p);
    if (st != CTP_OK)
        return st;
    return project_into(plan, vol, vol_dtype, sino, sino_dtype, batch, accumulate ? 1 : 0,
                        workspace, p, stream);
}

ctp_status ctp_project_static(const ctp_plan *plan, const void *vol, ctp_dtype vol_dtype,
                              void *sino, ctp_dtype sino_dtype, int64_t batch, int accumulate,
                              hipStream_t stream)
{
    g_last_error.clear();
    // the same checks as ctp_project, then the size of the call's workspace against the array
    size_t need = 0;
    ctp_status st = ctp_workspace_bytes(plan, CTP_FORWARD, vol_dtype, sino_dtype, batch, &need);
    if (st != CTP_OK)
        return st;
    if (need > ctp::kStaticScratchBytes)
        return fail(CTP_EINVAL, "call needs " + std::to_string(need) +
                                    " bytes of scratch; the static scratch holds " +
                                    std::to_string(ctp::kStaticScratchBytes) +
                                    " (use ctp_project with a workspace)");
    void *scratch = nullptr;
    const hipError_t e = ctp::static_scratch(&scratch);
    if (e != hipSuccess)
        return fail(CTP_EDEVICE, std::string("static scratch address: ") + hipGetErrorString(e));
    ctp::Params p;
    st = prepare_call(plan, vol, sino, vol_dtype, sino_dtype, batch, scratch,
                      ctp::kStaticScratchBytes, CTP_FORWARD, p);
    if (st != CTP_OK)
        return st;
    return project_into(plan, vol, vol_dtype, sino, sino_dtype, batch, accumulate ? 1 : 0,
                        scratch, p, stream);
}

}  // extern "C"

namespace {

// The back projection into a validated workspace (prepare_call has run), in launches of at most
// views_per_launch views (0: one launch): the first launch starts each voxel's sum, the later
// ones continue it, so every voxel adds its views in the same order as in a single launch.
ctp_status backproject_into(const ctp_plan *plan, const void *sino, ctp_dtype sino_dtype,
                            void *vol, ctp_dtype vol_dtype, int64_t batch, int accumulate,
                            void *workspace, ctp::Params p, hipStream_t stream,
                            int views_per_launch = 0)
{
    const BwdWs w = bwd_ws_layout(plan, batch, vol_dtype, sino_dtype);
    char *ws = static_cast<char *>(workspace);
    const float *ys = static_cast<const float *>(sino);
    hipError_t e = hipSuccess;
    if (w.scaled) {
        e = ctp::launch_amp_scale(p, plan->cfg, plan->d_views, sino, (int)sino_dtype,
                                  reinterpret_cast<float *>(ws + w.ysc_off), batch, stream);
        ys = reinterpret_cast<const float *>(ws + w.ysc_off);
    }
    const bool half_out = vol_dtype != CTP_F32;
    float *out = half_out ? reinterpret_cast<float *>(ws + w.vol_off) : static_cast<float *>(vol);
    const int nv = plan->g.n_views;
    const int step = views_per_launch > 0 ? std::min(views_per_launch, nv) : nv;
    if (step < nv && accumulate && !half_out)
        return fail(CTP_EINVAL, "a back projection split over launches cannot accumulate");
    for (int v0 = 0; v0 < nv && e == hipSuccess; v0 += step) {
        p.v_begin = v0;
        p.v_count = std::min(step, nv - v0);
        e = ctp::launch_backward(p, plan->cfg, plan->d_views, ys, out, batch,
                                 v0 > 0 ? 2 : half_out ? 0 : accumulate, stream);
    }
    if (e == hipSuccess && half_out) {
        size_t vb = 0;
        ctp_plan_bytes(plan, CTP_F32, batch, &vb, nullptr);
        e = ctp::launch_store_convert(out, vol, (int)vol_dtype, (int64_t)(vb / 4), accumulate, stream);
    }
    return finish(e, stream, "back projection");
}

}  // namespace

extern "C" {

ctp_status ctp_backproject(const ctp_plan *plan, const void *sino, ctp_dtype sino_dtype, void *vol,
                           ctp_dtype vol_dtype, int64_t batch, int accumulate, void *workspace,
                           size_t workspace_bytes, hipStream_t stream)
{
    g_last_error.clear();
    ctp::Params p;
    ctp_status st = prepare_call(plan, sino, vol, sino_dtype, vol_dtype, batch, workspace,
                                 workspace_bytes, CTP_BACKWARD, p);
    if (st != CTP_OK)
        return st;
    return backproject_into(plan, sino, sino_dtype, vol, vol_dtype, batch, accumulate ? 1 : 0,
                            workspace, p, stream);
}

}  // extern "C"

namespace ctp {

ctp_status project_sliced(const ctp_plan *plan, const void *vol, ctp_dtype vol_dtype, void *sino,
                          ctp_dtype sino_dtype, int64_t batch, void *workspace,
                          size_t workspace_bytes, int views_per_launch, hipStream_t stream)
{
    g_last_error.clear();
    if (views_per_launch < 1)
        return fail(CTP_EINVAL, "views_per_launch must be >= 1");
    Params p;
    ctp_status st = prepare_call(plan, vol, sino, vol_dtype, sino_dtype, batch, workspace,
                                 workspace_bytes, CTP_FORWARD, p);
    if (st != CTP_OK)
        return st;
    return project_into(plan, vol, vol_dtype, sino, sino_dtype, batch, 0, workspace, p, stream,
                        views_per_launch);
}

ctp_status backproject_sliced(const ctp_plan *plan, const void *sino, ctp_dtype sino_dtype,
                              void *vol, ctp_dtype vol_dtype, int64_t batch, void *workspace,
                              size_t workspace_bytes, int views_per_launch, hipStream_t stream)
{
    g_last_error.clear();
    if (views_per_launch < 1)
        return fail(CTP_EINVAL, "views_per_launch must be >= 1");
    Params p;
    ctp_status st = prepare_call(plan, sino, vol, sino_dtype, vol_dtype, batch, workspace,
                                 workspace_bytes, CTP_BACKWARD, p);
    if (st != CTP_OK)
        return st;
    return backproject_into(plan, sino, sino_dtype, vol, vol_dtype, batch, 0, workspace, p,
                            stream, views_per_launch);
}

}  // namespace ctp

extern "C" {

ctp_status ctp_ramp_filter(const ctp_plan *plan, const void *sino, ctp_dtype sino_dtype, void *out,
                           ctp_dtype out_dtype, int64_t batch, ctp_window window,
                           hipStream_t stream)
{
    g_last_error.clear();
    if (plan == nullptr || sino == nullptr || out == nullptr)
        return fail(CTP_EINVAL, "NULL plan or data pointer");
    if (batch < 1)
        return fail(CTP_EINVAL, "batch must be >= 1");
    for (ctp_dtype d : {sino_dtype, out_dtype})
        if (d != CTP_F32 && d != CTP_BF16 && d != CTP_F16)
            return fail(CTP_EINVAL, "unknown dtype");
    if (window != CTP_WINDOW_RAMLAK && window != CTP_WINDOW_SHEPP_LOGAN)
        return fail(CTP_EINVAL, "unknown window");
    if (plan->g.kind == CTP_CONE_NONCIRC)
        return fail(CTP_EUNSUPPORTED, "the ramp filter weighting is defined for circular scans");
    if (plan->g.nu > 5120)
        return fail(CTP_EUNSUPPORTED, "more than 5120 detector columns");
    if (plan->g.n_views > 65535)
        return fail(CTP_EUNSUPPORTED, "more than 65535 views");
    const bool two_d = plan->g.kind == CTP_FAN2D;
    if (!two_d && batch > 65535)
        return fail(CTP_EINVAL, "batch too large");
    size_t in_b = 0, out_b = 0;
    ctp_plan_bytes(plan, sino_dtype, batch, nullptr, &in_b);
    ctp_plan_bytes(plan, out_dtype, batch, nullptr, &out_b);
    const char *a0 = static_cast<const char *>(sino), *b0 = static_cast<const char *>(out);
    if (a0 == b0 ? sino_dtype != out_dtype : (a0 < b0 + out_b && b0 < a0 + in_b))
        return fail(CTP_EINVAL, "input and output overlap (only exact in-place with one type is allowed)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
        return fail(CTP_EINVAL, "plan was created on another device");
    ctp::Params p = plan->base;
    const ctp_geometry_desc &g = plan->g;
    if (two_d) {
        p.nz = (int)batch;
        p.nv = (int)batch;
        p.sino_row_stride = (int64_t)g.n_views * g.nu;
        p.sino_view_stride = g.nu;
        p.sino_b_stride = 0;
    } else {
        p.sino_row_stride = g.nu;
        p.sino_view_stride = (int64_t)g.nv * g.nu;
        p.sino_b_stride = (int64_t)g.n_views * g.nv * g.nu;
    }
    const float dbeta = (float)(2.0 * 3.14159265358979323846 / g.n_views);
    hipError_t e = ctp::launch_ramp(p, plan->cfg, plan->d_views, sino, (int)sino_dtype, out,
                                    (int)out_dtype, two_d ? 1 : batch, (int)window, dbeta, stream);
    return finish(e, stream, "ramp filter");
}

}  // extern "C"
