/*
 * ctoracle.c -- FP64 CPU oracle for the separable-footprint (SF) and distance-driven (DD)
 * CT projectors and their exact adjoints.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load or call this library.  It shares no code, header or table with
 * the HIP engine, and the engine never calls it.
 *
 * What it computes (paper: Section 2.3, Eqs. 1-2; Section 2.2 and Table 1 for geometry):
 *   forward   y = A x   (Eq. 1), A never stored, computed voxel by voxel;
 *   adjoint   x = A^T y (Eq. 2), the literal transpose of the same weights, so the pair is
 *             matched (Section 2.3: forward and back projection are each other's gradient).
 * SF is the volume-based (box) voxel model and DD the face-based one (Section 2.3).  The
 * paper cites both methods without writing their formulas; the steps below are written from
 * the box-voxel line-integral model, in the order the cited methods use:
 *   SF:  transaxial trapezoid from the four corner projections, axial trapezoid from the
 *        bottom/top faces (SF-TT), amplitude l_phi0 per voxel-view times a per-cell polar
 *        amplitude |r|/|r_xy| ("A2"), cell average by the trapezoid's antiderivative;
 *   DD:  per view a driving axis; detector cell edges mapped onto each voxel plane through
 *        the source; weight = fractional overlap in the plane x fractional overlap along z
 *        (rows mapped along the column-centre ray) x the ray's path through the slab.
 * "recon" mode (Section 2.3: the FBP back projection carries a depth-dependent weight) uses
 * the SF footprint normalised to unit sum as the interpolation kernel and weights each view by
 * (SAD / W)^2; its forward projection is the transpose (method code 2, circular scans).
 * Every point the paper leaves open is fixed by one reading; the readings are listed with
 * the design notes.  Everything is double precision, no fast-math, no reordering beyond
 * skipping cells that the footprint does not reach.
 *
 * Parity status: SF and DD forward/adjoint are pinned by the test suite (closed form of a
 * single voxel, parallel-beam exactness against exact path lengths, mass conservation,
 * adjoint identity and full-matrix gradient check, symmetries, reductions, brute-force ray
 * integration, analytic ellipsoids, empty/outside-FOV cases); every pose and offset parameter
 * of the geometry and the curved-detector mapping by closed-form projections of single voxels
 * and by brute force with the parameter set; the distance-driven row mapping by the mirror
 * symmetry of the curved detector.  A mutation test builds this file with one-line mistakes
 * (flipped signs, dropped terms, wrong formulas) and requires a pin to fail for each.  Recon
 * mode is pinned by the closed-form sum of its weights, the adjoint identity and filtered back
 * projection of analytic discs and balls.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- geometry description (per-view arrays are already broadcast to n_views) ---- */
typedef struct {
    int32_t kind;   /* 0 = 2D fan beam, 1 = 3D circular cone beam, 2 = 3D non-circular */
    int32_t det;    /* 0 = flat detector, 1 = curved (cylindrical arc centred on the source) */
    int32_t nx, ny, nz;
    double dx, dy, dz;
    int32_t nu, nv;
    double du, dv;
    int32_t n_views;
    const double *theta, *phi, *psi, *sad, *sdd, *x_src, *z_src,
                 *x_ofst, *y_ofst, *z_ofst, *u_ofst, *v_ofst;
} orc_geom;

/* One view's frame in world coordinates (Section 2.2, Table 1). */
typedef struct {
    double s[3];          /* source */
    double d[3];          /* detector reference point (centre before the u/v offsets) */
    double eu[3], ev[3];  /* detector axes */
    double n[3];          /* detector normal, pointing towards the source */
    double sdd;
    double u_first;       /* centre of column 0 (includes -u_ofst) */
    double v_first;       /* centre of row 0 (includes -v_ofst) */
    double o[3];          /* object centre */
} orc_frame;

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void matvec3(double R[3][3], const double a[3], double out[3])
{
    for (int r = 0; r < 3; ++r)
        out[r] = R[r][0] * a[0] + R[r][1] * a[1] + R[r][2] * a[2];
}

static void matmul3(double A[3][3], double B[3][3], double C[3][3])
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            C[r][c] = A[r][0] * B[0][c] + A[r][1] * B[1][c] + A[r][2] * B[2][c];
}

/*
 * Frame of view b.  At theta = 0 the source sits at (x_src, SAD, z_src), the detector
 * reference point at (0, SAD - SDD, 0), e_u = +x, e_v = +z and the normal n = +y.  The
 * gantry pose R = Rz(theta) Rx(phi) Ry(psi) (rotation about y first, then x, then z; each
 * counter-clockwise about its axis) is applied to all of them.  Circular scans use
 * phi = psi = 0.  The object centre (x_ofst, y_ofst, z_ofst) is a world position; it does
 * not rotate with the gantry.  Column i is centred at u = (i - (nu-1)/2) du - u_ofst, row j
 * at v = (j - (nv-1)/2) dv - v_ofst (Table 1: detector position (-u_ofst, -v_ofst)).
 */
static void make_frame(const orc_geom *g, int b, orc_frame *f)
{
    const int three_d = g->kind != 0;
    const double th = g->theta[b];
    const double ph = g->kind == 2 ? g->phi[b] : 0.0;
    const double ps = g->kind == 2 ? g->psi[b] : 0.0;
    double Rz[3][3] = {{cos(th), -sin(th), 0}, {sin(th), cos(th), 0}, {0, 0, 1}};
    double Rx[3][3] = {{1, 0, 0}, {0, cos(ph), -sin(ph)}, {0, sin(ph), cos(ph)}};
    double Ry[3][3] = {{cos(ps), 0, sin(ps)}, {0, 1, 0}, {-sin(ps), 0, cos(ps)}};
    double T[3][3], R[3][3];
    matmul3(Rx, Ry, T);
    matmul3(Rz, T, R);

    const double s0[3] = {g->x_src[b], g->sad[b], three_d ? g->z_src[b] : 0.0};
    const double d0[3] = {0.0, g->sad[b] - g->sdd[b], 0.0};
    const double ex[3] = {1, 0, 0}, ey[3] = {0, 1, 0}, ez[3] = {0, 0, 1};
    matvec3(R, s0, f->s);
    matvec3(R, d0, f->d);
    matvec3(R, ex, f->eu);
    matvec3(R, ez, f->ev);
    matvec3(R, ey, f->n);
    f->sdd = g->sdd[b];
    f->u_first = -0.5 * (g->nu - 1) * g->du - g->u_ofst[b];
    f->v_first = three_d ? -0.5 * (g->nv - 1) * g->dv - g->v_ofst[b] : 0.0;
    f->o[0] = g->x_ofst[b];
    f->o[1] = g->y_ofst[b];
    f->o[2] = three_d ? g->z_ofst[b] : 0.0;
}

/* Detector coordinates (u, v) of world point p.
 * Flat:   W = (s-p).n, D = (s-d).n, u = (s-d).e_u + D (p-s).e_u / W, same for v with e_v.
 * Curved: a = (p-s).e_u, w = (s-p).n, u = SDD atan2(a, w) (arc length at radius SDD),
 *         v = (s-d).e_v + SDD (p-s).e_v / sqrt(a^2 + w^2). */
static void project(const orc_geom *g, const orc_frame *f, const double p[3],
                    double *u, double *v)
{
    double ps[3], sd[3];
    for (int k = 0; k < 3; ++k) {
        ps[k] = p[k] - f->s[k];
        sd[k] = f->s[k] - f->d[k];
    }
    if (g->det == 0) {
        const double W = -dot3(ps, f->n);
        const double D = dot3(sd, f->n);
        *u = dot3(sd, f->eu) + D * dot3(ps, f->eu) / W;
        *v = dot3(sd, f->ev) + D * dot3(ps, f->ev) / W;
    } else {
        const double a = dot3(ps, f->eu);
        const double w = -dot3(ps, f->n);
        *u = f->sdd * atan2(a, w);
        *v = dot3(sd, f->ev) + f->sdd * dot3(ps, f->ev) / sqrt(a * a + w * w);
    }
}

/* World position of the detector point with detector coordinates (u, v). */
static void det_point(const orc_geom *g, const orc_frame *f, double u, double v, double out[3])
{
    if (g->det == 0) {
        for (int k = 0; k < 3; ++k)
            out[k] = f->d[k] + u * f->eu[k] + v * f->ev[k];
    } else {
        double sd[3];
        for (int k = 0; k < 3; ++k)
            sd[k] = f->s[k] - f->d[k];
        const double gam = u / f->sdd;
        const double h = v - dot3(sd, f->ev);
        for (int k = 0; k < 3; ++k)
            out[k] = f->s[k] + f->sdd * (sin(gam) * f->eu[k] - cos(gam) * f->n[k]) + h * f->ev[k];
    }
}

static void voxel_centre(const orc_geom *g, const orc_frame *f, int ix, int iy, int iz,
                         double c[3])
{
    c[0] = f->o[0] + (ix - 0.5 * (g->nx - 1)) * g->dx;
    c[1] = f->o[1] + (iy - 0.5 * (g->ny - 1)) * g->dy;
    c[2] = g->kind == 0 ? 0.0 : f->o[2] + (iz - 0.5 * (g->nz - 1)) * g->dz;
}

static void sort4(double t[4])
{
    for (int a = 1; a < 4; ++a) {
        double x = t[a];
        int b = a - 1;
        while (b >= 0 && t[b] > x) {
            t[b + 1] = t[b];
            --b;
        }
        t[b + 1] = x;
    }
}

/*
 * Antiderivative G(t) of the unit-height trapezoid with sorted corners t0 <= t1 <= t2 <= t3:
 * rises linearly on [t0, t1], equals 1 on [t1, t2], falls linearly on [t2, t3].  A ramp
 * narrower than eps is treated as a step (no division).
 */
static double trap_cdf(const double k[4], double t, double eps)
{
    const double r1 = k[1] - k[0], r2 = k[3] - k[2];
    if (t <= k[0])
        return 0.0;
    if (t <= k[1])
        return r1 > eps ? (t - k[0]) * (t - k[0]) / (2.0 * r1) : 0.0;
    const double g1 = r1 > eps ? 0.5 * r1 : 0.0;
    if (t <= k[2])
        return g1 + (t - k[1]);
    const double g2 = g1 + (k[2] - k[1]);
    if (t <= k[3])
        return r2 > eps ? g2 + 0.5 * r2 - (k[3] - t) * (k[3] - t) / (2.0 * r2) : g2;
    return g2 + (r2 > eps ? 0.5 * r2 : 0.0);
}

/* Range of cells [lo, hi] (clipped to [0, n-1]) that an interval (a, b) can touch on a grid
 * with first edge e0 and pitch h.  Returns 0 when no cell is touched. */
static int cell_range(double a, double b, double e0, double h, int n, int *lo, int *hi)
{
    double fa = floor((a - e0) / h), fb = floor((b - e0) / h);
    if (fb < 0.0 || fa > n - 1)
        return 0;
    *lo = fa < 0.0 ? 0 : (int)fa;
    *hi = fb > n - 1 ? n - 1 : (int)fb;
    return *hi >= *lo;
}

/* ------------------------------------------------------------------------------------ */
/*  Separable footprint                                                                  */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    int i0, ni, j0, nj;   /* touched columns / rows */
    double amp;           /* l_phi0 */
    double *F1;           /* [ni] cell-averaged transaxial trapezoid */
    double *F2;           /* [nj] cell-averaged axial trapezoid (3D) */
    double Au, Av;        /* areas of the unit-height trapezoids in cells (sum of F1 / F2 over an
                             unbounded detector); Av = 1 in 2D */
    double W;             /* depth of the voxel centre: flat (s - c).n, curved the in-plane
                             distance from the source */
} sf_fp;

/*
 * SF footprint of voxel (ix, iy, iz) in view f.
 *   tau   = sorted u-projections of the four transaxial corners c +- dx/2 x +- dy/2 y, taken
 *           in the voxel's mid-plane z = c_z;
 *   kappa = sorted {min, max} of the v-projections of the four bottom corners and {min, max}
 *           of the four top corners (SF-TT);
 *   l     = min(dx/|g_x|, dy/|g_y|), g the unit xy-direction from the source to the centre;
 *   F1_i  = [G_tau(u_i + du/2) - G_tau(u_i - du/2)] / du, F2_j likewise along v.
 * Returns 0 when the footprint misses the detector.
 */
static int sf_footprint(const orc_geom *g, const orc_frame *f, int ix, int iy, int iz, sf_fp *fp)
{
    double c[3], p[3], tau[4], u, v;
    voxel_centre(g, f, ix, iy, iz, c);
    const double hx = 0.5 * g->dx, hy = 0.5 * g->dy, hz = 0.5 * g->dz;
    const double sx[4] = {-1, 1, -1, 1}, sy[4] = {-1, -1, 1, 1};

    for (int k = 0; k < 4; ++k) {
        p[0] = c[0] + sx[k] * hx;
        p[1] = c[1] + sy[k] * hy;
        p[2] = c[2];
        project(g, f, p, &u, &v);
        tau[k] = u;
    }
    sort4(tau);

    const double ue0 = f->u_first - 0.5 * g->du;
    if (!cell_range(tau[0], tau[3], ue0, g->du, g->nu, &fp->i0, &fp->ni))
        return 0;
    fp->ni = fp->ni - fp->i0 + 1;

    if (g->kind != 0) {
        double kap[4];
        double bmin = INFINITY, bmax = -INFINITY, tmin = INFINITY, tmax = -INFINITY;
        for (int k = 0; k < 4; ++k) {
            p[0] = c[0] + sx[k] * hx;
            p[1] = c[1] + sy[k] * hy;
            p[2] = c[2] - hz;
            project(g, f, p, &u, &v);
            bmin = fmin(bmin, v);
            bmax = fmax(bmax, v);
            p[2] = c[2] + hz;
            project(g, f, p, &u, &v);
            tmin = fmin(tmin, v);
            tmax = fmax(tmax, v);
        }
        kap[0] = bmin;
        kap[1] = bmax;
        kap[2] = tmin;
        kap[3] = tmax;
        sort4(kap);
        fp->Av = 0.5 * (kap[3] + kap[2] - kap[1] - kap[0]) / g->dv;
        const double ve0 = f->v_first - 0.5 * g->dv;
        if (!cell_range(kap[0], kap[3], ve0, g->dv, g->nv, &fp->j0, &fp->nj))
            return 0;
        fp->nj = fp->nj - fp->j0 + 1;
        for (int j = 0; j < fp->nj; ++j) {
            const double e = ve0 + (fp->j0 + j) * g->dv;
            fp->F2[j] = (trap_cdf(kap, e + g->dv, 1e-12 * g->dv) - trap_cdf(kap, e, 1e-12 * g->dv)) / g->dv;
        }
    } else {
        fp->j0 = 0;
        fp->nj = 1;
        fp->F2[0] = 1.0;
        fp->Av = 1.0;
    }
    fp->Au = 0.5 * (tau[3] + tau[2] - tau[1] - tau[0]) / g->du;
    {
        const double w = (f->s[0] - c[0]) * f->n[0] + (f->s[1] - c[1]) * f->n[1] +
                         (f->s[2] - c[2]) * f->n[2];
        if (g->det == 1) {
            const double a = (c[0] - f->s[0]) * f->eu[0] + (c[1] - f->s[1]) * f->eu[1] +
                             (c[2] - f->s[2]) * f->eu[2];
            fp->W = sqrt(a * a + w * w);
        } else {
            fp->W = w;
        }
    }

    for (int i = 0; i < fp->ni; ++i) {
        const double e = ue0 + (fp->i0 + i) * g->du;
        fp->F1[i] = (trap_cdf(tau, e + g->du, 1e-12 * g->du) - trap_cdf(tau, e, 1e-12 * g->du)) / g->du;
    }

    const double gx = c[0] - f->s[0], gy = c[1] - f->s[1];
    const double nrm = hypot(gx, gy);
    const double lx = gx != 0.0 ? g->dx * nrm / fabs(gx) : INFINITY;
    const double ly = gy != 0.0 ? g->dy * nrm / fabs(gy) : INFINITY;
    fp->amp = fmin(lx, ly);
    return 1;
}

/* Per-cell SF amplitude (reading "A2"): |r| / |r_xy|, r = centre of cell (i, j) - source.
 * In 2D it is 1. */
static double sf_cell_amp(const orc_geom *g, const orc_frame *f, int i, int j)
{
    if (g->kind == 0)
        return 1.0;
    double q[3];
    det_point(g, f, f->u_first + i * g->du, f->v_first + j * g->dv, q);
    const double rx = q[0] - f->s[0], ry = q[1] - f->s[1], rz = q[2] - f->s[2];
    return sqrt(rx * rx + ry * ry + rz * rz) / hypot(rx, ry);
}

/*
 * "recon" mode (Section 2.3: the back projection of FBP carries a depth-dependent weight).
 * The voxel's SF footprint serves as an interpolation kernel normalised to unit sum,
 * F1_i F2_j / (Au Av), and each view is weighted by (SAD / W)^2 with W the voxel centre's
 * depth (flat: distance along the detector normal; curved: in-plane distance from the source),
 * the 1/U^2 factor of fan-beam and cone-beam FBP.  No per-cell amplitude.  The forward
 * projection in this mode is the transpose of that back projection.
 */
static double sf_recon_weight(const orc_geom *g, int b, const sf_fp *fp)
{
    const double r = g->sad[b] / fp->W;
    return r * r / (fp->Au * fp->Av);
}

/* ------------------------------------------------------------------------------------ */
/*  Distance driven                                                                      */
/* ------------------------------------------------------------------------------------ */

/* Driving axis of a view: y (planes y = const) when |n_y| >= |n_x|, else x. */
static int dd_y_driven(const orc_frame *f)
{
    return fabs(f->n[1]) >= fabs(f->n[0]);
}

/* Coordinate along the in-plane axis where the source ray through detector point q meets the
 * driving plane (coordinate `plane` along the driving axis); also returns the ray parameter
 * t (0 at the source, 1 at q). */
static double dd_map(const orc_frame *f, const double q[3], int ydrv, double plane, double *t)
{
    const int a = ydrv ? 1 : 0, b = ydrv ? 0 : 1;
    *t = (plane - f->s[a]) / (q[a] - f->s[a]);
    return f->s[b] + *t * (q[b] - f->s[b]);
}

typedef struct {
    int i0, ni;           /* touched columns */
    double *Fx;           /* [ni] transaxial overlap fraction */
    int *j0, *nj;         /* [ni] touched rows per column */
    double *Fz;           /* [ni * nv] axial overlap fraction, row-major by column */
} dd_fp;

/*
 * DD footprint of voxel (ix, iy, iz) in view f (circular geometries only).
 * y-driven: the voxel's plane is y = c_y and its in-plane interval [c_x -+ dx/2]; each column
 * edge u is mapped to X(u) on that plane along the source ray; Fx_i = overlap of the voxel
 * interval with [X(u_i - du/2), X(u_i + du/2)] divided by that mapped width.
 * Axially (3D), the rows of column i are mapped along the ray through the column centre:
 * Z(v) = s_z + t_i (q_z(v) - s_z); Fz_ij = overlap of [c_z -+ dz/2] with the mapped row,
 * divided by the mapped row height.  x-driven views swap the roles of x and y.
 */
static int dd_footprint(const orc_geom *g, const orc_frame *f, int ix, int iy, int iz, dd_fp *fp)
{
    double c[3], p[3], q[3], t, u, v;
    voxel_centre(g, f, ix, iy, iz, c);
    const int yd = dd_y_driven(f);
    const double plane = yd ? c[1] : c[0];
    const double lo = yd ? c[0] - 0.5 * g->dx : c[1] - 0.5 * g->dy;
    const double hi = yd ? c[0] + 0.5 * g->dx : c[1] + 0.5 * g->dy;

    /* columns touched: project the two in-plane edge points of the voxel */
    double ua, ub;
    p[2] = c[2];
    if (yd) { p[0] = lo; p[1] = plane; } else { p[0] = plane; p[1] = lo; }
    project(g, f, p, &ua, &v);
    if (yd) { p[0] = hi; p[1] = plane; } else { p[0] = plane; p[1] = hi; }
    project(g, f, p, &ub, &v);
    const double ue0 = f->u_first - 0.5 * g->du;
    int i_lo, i_hi;
    if (!cell_range(fmin(ua, ub), fmax(ua, ub), ue0, g->du, g->nu, &i_lo, &i_hi))
        return 0;
    fp->i0 = i_lo;
    fp->ni = i_hi - i_lo + 1;

    const double ve0 = f->v_first - 0.5 * g->dv;
    for (int k = 0; k < fp->ni; ++k) {
        const int i = i_lo + k;
        det_point(g, f, ue0 + i * g->du, 0.0, q);
        const double Xa = dd_map(f, q, yd, plane, &t);
        det_point(g, f, ue0 + (i + 1) * g->du, 0.0, q);
        const double Xb = dd_map(f, q, yd, plane, &t);
        const double mlo = fmin(Xa, Xb), mhi = fmax(Xa, Xb);
        const double ov = fmin(hi, mhi) - fmax(lo, mlo);
        fp->Fx[k] = ov > 0.0 ? ov / (mhi - mlo) : 0.0;

        if (g->kind == 0) {
            fp->j0[k] = 0;
            fp->nj[k] = 1;
            fp->Fz[k * g->nv] = 1.0;
            continue;
        }
        /* axial map along the column-centre ray */
        det_point(g, f, f->u_first + i * g->du, 0.0, q);
        dd_map(f, q, yd, plane, &t);
        const double zlo = c[2] - 0.5 * g->dz, zhi = c[2] + 0.5 * g->dz;
        /* rows touched: invert Z(v) at the voxel's z-limits */
        double qa[3], qb[3];
        det_point(g, f, f->u_first + i * g->du, ve0, qa);
        det_point(g, f, f->u_first + i * g->du, ve0 + g->dv, qb);
        const double za0 = f->s[2] + t * (qa[2] - f->s[2]);
        const double zslope = t * (qb[2] - qa[2]);        /* mapped height of one row */
        int j_lo, j_hi;
        if (!cell_range(fmin((zlo - za0) / zslope, (zhi - za0) / zslope),
                        fmax((zlo - za0) / zslope, (zhi - za0) / zslope),
                        0.0, 1.0, g->nv, &j_lo, &j_hi)) {
            fp->j0[k] = 0;
            fp->nj[k] = 0;
            continue;
        }
        fp->j0[k] = j_lo;
        fp->nj[k] = j_hi - j_lo + 1;
        for (int j = j_lo; j <= j_hi; ++j) {
            det_point(g, f, f->u_first + i * g->du, ve0 + j * g->dv, qa);
            det_point(g, f, f->u_first + i * g->du, ve0 + (j + 1) * g->dv, qb);
            const double Za = f->s[2] + t * (qa[2] - f->s[2]);
            const double Zb = f->s[2] + t * (qb[2] - f->s[2]);
            const double rlo = fmin(Za, Zb), rhi = fmax(Za, Zb);
            const double oz = fmin(zhi, rhi) - fmax(zlo, rlo);
            fp->Fz[k * g->nv + (j - j_lo)] = oz > 0.0 ? oz / (rhi - rlo) : 0.0;
        }
    }
    (void)u;
    return 1;
}

/* Per-cell DD amplitude: slab thickness along the driving axis times |rho| / |rho_drive|,
 * rho = centre of cell (i, j) - source. */
static double dd_cell_amp(const orc_geom *g, const orc_frame *f, int i, int j)
{
    double q[3];
    det_point(g, f, f->u_first + i * g->du, g->kind == 0 ? 0.0 : f->v_first + j * g->dv, q);
    const double rx = q[0] - f->s[0], ry = q[1] - f->s[1];
    const double rz = g->kind == 0 ? 0.0 : q[2] - f->s[2];
    const double r = sqrt(rx * rx + ry * ry + rz * rz);
    return dd_y_driven(f) ? g->dy * r / fabs(ry) : g->dx * r / fabs(rx);
}

/* ------------------------------------------------------------------------------------ */
/*  Public entry points                                                                  */
/* ------------------------------------------------------------------------------------ */

static int check_geom(const orc_geom *g, int method)
{
    if (g->kind < 0 || g->kind > 2 || g->det < 0 || g->det > 1 || method < 0 || method > 2)
        return -1;
    if (method == 2 && g->kind == 2)
        return -2;          /* recon mode: circular scans (FBP / FDK) */
    if (g->kind == 2 && g->det == 1)
        return -2;          /* non-circular geometries use flat detectors only */
    if (method == 1 && g->kind == 2)
        return -2;          /* DD is built for circular geometries */
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->nu <= 0 || g->nv <= 0 || g->n_views <= 0)
        return -1;
    return 0;
}

static int64_t vol_index(const orc_geom *g, int ix, int iy, int iz)
{
    return ((int64_t)iz * g->ny + iy) * g->nx + ix;
}

static int nz_of(const orc_geom *g) { return g->kind == 0 ? 1 : g->nz; }
static int nv_of(const orc_geom *g) { return g->kind == 0 ? 1 : g->nv; }

/* Forward projection of one volume for the listed views.
 * vol:  [nz][ny][nx] (nz = 1 in 2D);  sino: [n_list][nv][nu] (nv = 1 in 2D), overwritten.
 * method: 0 = SF, 1 = DD, 2 = SF in "recon" mode (the transpose of the FBP back projection,
 * see sf_recon_weight).  Returns 0 on success, <0 on an unsupported/invalid geometry. */
int orc_forward(const orc_geom *g, int method, const double *vol, int n_list, const int32_t *views,
                double *sino)
{
    int rc = check_geom(g, method);
    if (rc)
        return rc;
    const int nz = nz_of(g), nv = nv_of(g), nu = g->nu;
    const int64_t view_sz = (int64_t)nv * nu;

#pragma omp parallel
    {
        double *F1 = malloc(sizeof(double) * (size_t)nu);
        double *F2 = malloc(sizeof(double) * (size_t)nv);
        double *Fz = malloc(sizeof(double) * (size_t)nu * nv);
        int *j0 = malloc(sizeof(int) * (size_t)nu), *nj = malloc(sizeof(int) * (size_t)nu);
#pragma omp for schedule(dynamic, 1)
        for (int vi = 0; vi < n_list; ++vi) {
            orc_frame f;
            make_frame(g, views[vi], &f);
            double *y = sino + (int64_t)vi * view_sz;
            memset(y, 0, sizeof(double) * (size_t)view_sz);
            for (int iz = 0; iz < nz; ++iz)
                for (int iy = 0; iy < g->ny; ++iy)
                    for (int ix = 0; ix < g->nx; ++ix) {
                        const double x = vol[vol_index(g, ix, iy, iz)];
                        if (x == 0.0)
                            continue;
                        if (method != 1) {
                            sf_fp fp = {0, 0, 0, 0, 0.0, F1, F2, 0.0, 0.0, 0.0};
                            if (!sf_footprint(g, &f, ix, iy, iz, &fp))
                                continue;
                            const double amp = method == 2 ? sf_recon_weight(g, views[vi], &fp) : fp.amp;
                            for (int j = 0; j < fp.nj; ++j)
                                for (int i = 0; i < fp.ni; ++i)
                                    y[(int64_t)(fp.j0 + j) * nu + fp.i0 + i] += x * amp * fp.F1[i] * fp.F2[j];
                        } else {
                            dd_fp fp = {0, 0, F1, j0, nj, Fz};
                            if (!dd_footprint(g, &f, ix, iy, iz, &fp))
                                continue;
                            for (int k = 0; k < fp.ni; ++k)
                                for (int j = 0; j < fp.nj[k]; ++j)
                                    y[(int64_t)(fp.j0[k] + j) * nu + fp.i0 + k] += x * fp.Fx[k] * fp.Fz[k * nv + j];
                        }
                    }
            for (int j = 0; j < nv; ++j)
                for (int i = 0; i < nu; ++i)
                    y[(int64_t)j * nu + i] *= method == 0 ? sf_cell_amp(g, &f, i, j)
                                              : method == 1 ? dd_cell_amp(g, &f, i, j) : 1.0;
        }
        free(F1);
        free(F2);
        free(Fz);
        free(j0);
        free(nj);
    }
    return 0;
}

/* Adjoint (back projection) evaluated at the listed voxels (linear indices into
 * [nz][ny][nx]).  sino: [n_views][nv][nu]; out: [n_list].  The per-cell amplitude is applied
 * to the sinogram first (x = B^T diag(L) y), then the same footprint weights as the forward
 * projection are gathered. */
int orc_adjoint(const orc_geom *g, int method, const double *sino, int64_t n_list,
                const int64_t *voxels, double *out)
{
    int rc = check_geom(g, method);
    if (rc)
        return rc;
    const int nv = nv_of(g), nu = g->nu;
    const int64_t view_sz = (int64_t)nv * nu;
    const int64_t total = view_sz * g->n_views;
    double *ys = malloc(sizeof(double) * (size_t)total);
    orc_frame *fr = malloc(sizeof(orc_frame) * (size_t)g->n_views);
    if (!ys || !fr) {
        free(ys);
        free(fr);
        return -3;
    }
    for (int b = 0; b < g->n_views; ++b)
        make_frame(g, b, &fr[b]);

#pragma omp parallel for schedule(static)
    for (int b = 0; b < g->n_views; ++b)
        for (int j = 0; j < nv; ++j)
            for (int i = 0; i < nu; ++i) {
                const int64_t k = b * view_sz + (int64_t)j * nu + i;
                ys[k] = sino[k] * (method == 0 ? sf_cell_amp(g, &fr[b], i, j)
                                   : method == 1 ? dd_cell_amp(g, &fr[b], i, j) : 1.0);
            }

#pragma omp parallel
    {
        double *F1 = malloc(sizeof(double) * (size_t)nu);
        double *F2 = malloc(sizeof(double) * (size_t)nv);
        double *Fz = malloc(sizeof(double) * (size_t)nu * nv);
        int *j0 = malloc(sizeof(int) * (size_t)nu), *nj = malloc(sizeof(int) * (size_t)nu);
#pragma omp for schedule(dynamic, 64)
        for (int64_t n = 0; n < n_list; ++n) {
            const int64_t lin = voxels[n];
            const int ix = (int)(lin % g->nx);
            const int iy = (int)((lin / g->nx) % g->ny);
            const int iz = (int)(lin / ((int64_t)g->nx * g->ny));
            double acc = 0.0;
            for (int b = 0; b < g->n_views; ++b) {
                const double *y = ys + b * view_sz;
                if (method != 1) {
                    sf_fp fp = {0, 0, 0, 0, 0.0, F1, F2, 0.0, 0.0, 0.0};
                    if (!sf_footprint(g, &fr[b], ix, iy, iz, &fp))
                        continue;
                    const double amp = method == 2 ? sf_recon_weight(g, b, &fp) : fp.amp;
                    for (int j = 0; j < fp.nj; ++j)
                        for (int i = 0; i < fp.ni; ++i)
                            acc += amp * fp.F1[i] * fp.F2[j] * y[(int64_t)(fp.j0 + j) * nu + fp.i0 + i];
                } else {
                    dd_fp fp = {0, 0, F1, j0, nj, Fz};
                    if (!dd_footprint(g, &fr[b], ix, iy, iz, &fp))
                        continue;
                    for (int k = 0; k < fp.ni; ++k)
                        for (int j = 0; j < fp.nj[k]; ++j)
                            acc += fp.Fx[k] * fp.Fz[k * nv + j] * y[(int64_t)(fp.j0[k] + j) * nu + fp.i0 + k];
                }
            }
            out[n] = acc;
        }
        free(F1);
        free(F2);
        free(Fz);
        free(j0);
        free(nj);
    }
    free(ys);
    free(fr);
    return 0;
}

/* Counts for the listed views: voxel-views whose footprint meets the detector, non-zeros of A
 * (touched (voxel, cell) pairs), touched columns and rows.  out[0..3]. */
int orc_count(const orc_geom *g, int method, int n_list, const int32_t *views, int64_t *out)
{
    int rc = check_geom(g, method);
    if (rc)
        return rc;
    const int nz = nz_of(g), nv = nv_of(g), nu = g->nu;
    int64_t vv = 0, nnz = 0, cols = 0, rows = 0;
#pragma omp parallel reduction(+ : vv, nnz, cols, rows)
    {
        double *F1 = malloc(sizeof(double) * (size_t)nu);
        double *F2 = malloc(sizeof(double) * (size_t)nv);
        double *Fz = malloc(sizeof(double) * (size_t)nu * nv);
        int *j0 = malloc(sizeof(int) * (size_t)nu), *nj = malloc(sizeof(int) * (size_t)nu);
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int vi = 0; vi < n_list; ++vi)
            for (int iz = 0; iz < nz; ++iz) {
                orc_frame f;
                make_frame(g, views[vi], &f);
                for (int iy = 0; iy < g->ny; ++iy)
                    for (int ix = 0; ix < g->nx; ++ix) {
                        if (method != 1) {
                            sf_fp fp = {0, 0, 0, 0, 0.0, F1, F2, 0.0, 0.0, 0.0};
                            if (!sf_footprint(g, &f, ix, iy, iz, &fp))
                                continue;
                            vv += 1;
                            nnz += (int64_t)fp.ni * fp.nj;
                            cols += fp.ni;
                            rows += fp.nj;
                        } else {
                            dd_fp fp = {0, 0, F1, j0, nj, Fz};
                            if (!dd_footprint(g, &f, ix, iy, iz, &fp))
                                continue;
                            vv += 1;
                            cols += fp.ni;
                            for (int k = 0; k < fp.ni; ++k) {
                                nnz += fp.nj[k];
                                rows += fp.nj[k];
                            }
                        }
                    }
            }
        free(F1);
        free(F2);
        free(Fz);
        free(j0);
        free(nj);
    }
    out[0] = vv;
    out[1] = nnz;
    out[2] = cols;
    out[3] = rows;
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
