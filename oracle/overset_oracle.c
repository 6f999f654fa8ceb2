/*
 * Plain FP64 CPU oracle for the overset grid-assembly path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do. It shares no code with the HIP library.
 *
 * Method: Hedayat & Borazjani, "A parallel dynamic overset grid framework for
 * immersed boundary methods" (arXiv:1910.09315), Sec. 2.2 (grid assembly).
 * Every stage is written as the plain definition of what the paper's stage
 * computes, in FP64, built with -ffp-contract=off and a fixed evaluation order:
 *
 *   orc_transform      rigid frame map x = R X + c            (Sec. 2.1, frame of Fig. "non-inertial")
 *   orc_holecut        explicit hole cutting against closed blank surfaces
 *                      given as input: implicit shapes, or a closed surface
 *                      triangulation tested by ray parity      (Sec. 2.2.2)
 *   orc_mesh_inside    that ray-parity test for given points
 *   orc_fringe         potential query points: overset boundary faces and the
 *                      buffer layer around blanked nodes      (Sec. 2.2.3, item 1)
 *   orc_compact        the ordered query list and its count NQ (Sec. 2.2.3, Alg. 1)
 *   orc_bins_build     control cells: an axis-aligned auxiliary Cartesian grid
 *                      over the donor grid, each control cell listing the
 *                      donor cells that can reach it           (Sec. 2.2.5, AABB + control cells)
 *   orc_donor_search   brute-force search of the control cell (the paper's
 *                      fallback, Sec. 2.2.5 / Alg. 3) with containment decided by
 *                      trilinear natural coordinates found by Newton's method;
 *                      donor priority of Sec. 2.4 item 1; blanked donors invalid
 *   orc_interp         trilinear interpolation (Sec. 2.2.6)
 *   orc_frame_velocity interpolated velocity given in the receiver's frame
 *                      (Sec. 2.3, the non-inertial velocity relation)
 *   orc_interp_matrix  the interpolation matrix: per query the global indices
 *                      of its donor's corners and their weights (Sec. 2.2.6,
 *                      second option; Alg. 4)
 *   orc_matrix_apply   that matrix times field vectors
 *
 * The walk of Alg. 3 is an accelerator that must reach the same cell; the
 * oracle therefore omits it and searches every candidate cell.
 *
 * Readings of the paper that this file fixes (each is also listed with the
 * design notes):
 *  - flag byte: state in bits 0-1 (0 field, 1 hole, 2 fringe), cause grid in
 *    bits 2-7 (63 = overset outer boundary); hole > fringe > field.
 *  - hole test is the sign of an implicit closed surface, strict inside; a
 *    triangulated closed surface is tested by ray parity along +x with the
 *    edge rule of mesh_inside.
 *  - buffer layer = the non-hole nodes within Chebyshev index distance nf of a
 *    hole (outside the hole, 26-connected); cause = min over the causes met.
 *  - donor = the lowest linear cell index among valid containing cells of the
 *    first candidate grid that has one; candidates: the cause grid, then the
 *    background (grid 0), then the other grids in ascending id.
 *  - trilinear weights w_c = prod_d (c_d ? s_d : 1 - s_d), s measured from the
 *    lower-index face (the printed formula's signs are read this way).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ST_FIELD 0
#define ST_HOLE 1
#define ST_FRINGE 2
#define CAUSE_BOUNDARY 63

#define BLANK_NONE 0
#define BLANK_CYL 1
#define BLANK_SPHERE 2
#define BLANK_ELLIPSOID 3
#define BLANK_MESH 4

#define NEWTON_MAXIT 50
#define NEWTON_TOL 1e-12   /* stop when the last Newton step is this small */
#define S_TOL 1e-12        /* containment: s in [-S_TOL, 1 + S_TOL]^3 */
#define DET_MIN 1e-300

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* The thread count of the following parallel regions (n >= 1; timing only). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------ transform */
/* x_i = ((R_i0 X + R_i1 Y) + R_i2 Z) + c_i ; pose = R row-major (9) then c (3). */
static void apply_pose(const double *p, double X, double Y, double Z, double out[3]) {
    for (int i = 0; i < 3; ++i) {
        double a = p[3 * i + 0] * X;
        a = a + p[3 * i + 1] * Y;
        a = a + p[3 * i + 2] * Z;
        out[i] = a + p[9 + i];
    }
}

/* xi_i = ((R_0i d0 + R_1i d1) + R_2i d2), d = x - c : the inverse rigid map. */
static void apply_pose_inv(const double *p, const double x[3], double xi[3]) {
    double d0 = x[0] - p[9], d1 = x[1] - p[10], d2 = x[2] - p[11];
    for (int i = 0; i < 3; ++i) {
        double a = p[0 + i] * d0;
        a = a + p[3 + i] * d1;
        a = a + p[6 + i] * d2;
        xi[i] = a;
    }
}

void orc_transform(const double *pose, const double *X, const double *Y, const double *Z,
                   const int32_t *idx, int64_t n, double *x, double *y, double *z) {
    for (int64_t q = 0; q < n; ++q) {
        int64_t m = idx ? idx[q] : q;
        double w[3];
        apply_pose(pose, X[m], Y[m], Z[m], w);
        x[q] = w[0];
        y[q] = w[1];
        z[q] = w[2];
    }
}

/* ------------------------------------------------------------ hole cut */
/* Inside test of a blank region given by an implicit closed surface in the
 * body frame of its grid (the paper's user-defined closed blank surface,
 * Sec. 2.2.2; the sign of the implicit function replaces ray parity).
 * *gap receives a scale-free distance of xi from the surface, for diagnostics. */
static int blank_inside(int kind, const double *prm, const double xi[3], double *gap) {
    if (kind == BLANK_CYL) {               /* prm: r, z0, z1 */
        double r2 = prm[0] * prm[0];
        double rho2 = xi[0] * xi[0] + xi[1] * xi[1];
        double g = fabs(rho2 - r2) / r2;
        double gz0 = fabs(xi[2] - prm[1]) / prm[0], gz1 = fabs(xi[2] - prm[2]) / prm[0];
        if (gz0 < g) g = gz0;
        if (gz1 < g) g = gz1;
        *gap = g;
        return rho2 < r2 && xi[2] >= prm[1] && xi[2] <= prm[2];
    }
    if (kind == BLANK_SPHERE) {            /* prm: r */
        double r2 = prm[0] * prm[0];
        double rho2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        *gap = fabs(rho2 - r2) / r2;
        return rho2 < r2;
    }
    if (kind == BLANK_ELLIPSOID) {         /* prm: a, b, c */
        double u = xi[0] / prm[0], v = xi[1] / prm[1], w = xi[2] / prm[2];
        double f = u * u + v * v + w * w;
        *gap = fabs(f - 1.0);
        return f < 1.0;
    }
    *gap = INFINITY;
    return 0;
}

/* Inside test of a closed triangulated surface by ray parity (the hole cut
 * against the body's surface triangulation of Sec. 2.2.2): the ray from xi
 * along +x crosses the surface an odd number of times.
 *  - A triangle is crossed when xi's projection (y, z) lies in the
 *    triangle's projection and the crossing lies beyond xi in x.
 *  - The projection is taken counter-clockwise (b and c swapped when its
 *    signed area is negative; an edge-on triangle, area 0, is skipped).
 *  - Edge function of edge u->v at p: (v_y - u_y)(p_z - u_z) - (v_z - u_z)(p_y - u_y),
 *    computed from the endpoint with the smaller (y, z) (negated when that
 *    is v), so that it is exactly antisymmetric in u and v.
 *    p is in the projection when every edge function is > 0, or = 0 on an
 *    edge that is included: v_z > u_z, or v_z = u_z and v_y > u_y. An edge
 *    shared by two triangles on opposite sides is included by exactly one
 *    of them, so a crossing through a projected edge or vertex counts once.
 *  - The crossing is beyond xi when w0 a_x + w1 b_x + w2 c_x > x (w0 + w1 + w2),
 *    with the edge functions w opposite a, b, c (barycentric weights times
 *    the area, which is positive).
 * Outside the surface's axis-aligned box the point is outside. *gap
 * receives the smallest |crossing x - xi_x| met (diagnostic). */
static int edge_included(const double *u, const double *v) {
    double dz = v[2] - u[2], dy = v[1] - u[1];
    return dz > 0.0 || (dz == 0.0 && dy > 0.0);
}

static double edge_fn_raw(const double *u, const double *v, const double *p) {
    double t0 = (v[1] - u[1]) * (p[2] - u[2]);
    double t1 = (v[2] - u[2]) * (p[1] - u[1]);
    return t0 - t1;
}

/* Evaluated with the endpoints in a fixed order (ascending (y, z)) and
 * negated for the other direction, so that the two triangles sharing an
 * edge get exactly opposite values: rounding cannot put a point inside both
 * or neither. */
static double edge_fn(const double *u, const double *v, const double *p) {
    if (u[1] < v[1] || (u[1] == v[1] && u[2] < v[2])) return edge_fn_raw(u, v, p);
    return -edge_fn_raw(v, u, p);
}

static void mesh_box(const double *tri, int64_t ntri, double box[6]) {
    for (int d = 0; d < 3; ++d) {
        box[d] = INFINITY;
        box[3 + d] = -INFINITY;
    }
    for (int64_t k = 0; k < 3 * ntri; ++k)
        for (int d = 0; d < 3; ++d) {
            double v = tri[3 * k + d];
            if (v < box[d]) box[d] = v;
            if (v > box[3 + d]) box[3 + d] = v;
        }
}

static int mesh_inside(const double *tri, int64_t ntri, const double box[6], const double xi[3], double *gap) {
    *gap = INFINITY;
    for (int d = 0; d < 3; ++d)
        if (xi[d] < box[d] || xi[d] > box[3 + d]) return 0;
    int odd = 0;
    for (int64_t k = 0; k < ntri; ++k) {
        const double *a = tri + 9 * k, *b = a + 3, *c = a + 6;
        double area = edge_fn(a, b, c);
        if (area == 0.0) continue;
        if (area < 0.0) {
            const double *t = b;
            b = c;
            c = t;
        }
        double w0 = edge_fn(b, c, xi), w1 = edge_fn(c, a, xi), w2 = edge_fn(a, b, xi);
        if (!(w0 > 0.0 || (w0 == 0.0 && edge_included(b, c)))) continue;
        if (!(w1 > 0.0 || (w1 == 0.0 && edge_included(c, a)))) continue;
        if (!(w2 > 0.0 || (w2 == 0.0 && edge_included(a, b)))) continue;
        double den = (w0 + w1) + w2;
        double num = (w0 * a[0] + w1 * b[0]) + w2 * c[0];
        double rhs = xi[0] * den;
        double g = fabs(num - rhs) / den;
        if (g < *gap) *gap = g;
        if (num > rhs) odd ^= 1;
    }
    return odd;
}

/* The ray-parity test for n points xi[3n] against one surface; out[n] = 0/1.
 * Returns the smallest crossing gap met. */
double orc_mesh_inside(const double *tri, int64_t ntri, int64_t n, const double *xi, uint8_t *out) {
    double box[6], gmin = INFINITY;
    mesh_box(tri, ntri, box);
    for (int64_t q = 0; q < n; ++q) {
        double g;
        out[q] = (uint8_t)mesh_inside(tri, ntri, box, xi + 3 * q, &g);
        if (g < gmin) gmin = g;
    }
    return gmin;
}

/* dims: [ngrids*4] = ni, nj, nk, periodic ; coords: arrays of ngrids pointers ;
 * blank_prm: [ngrids*8] ; poses: [ngrids*12] ; node_off: [ngrids+1] ;
 * mesh_tri / mesh_ntri: per grid the triangles (9 doubles each, body frame)
 * of a BLANK_MESH region (NULL / 0 otherwise; both arrays may be NULL when
 * no grid has one). flags (total nodes) receives hole/field states. Returns
 * the smallest surface gap met (diagnostic: a tiny gap means the decision
 * is fragile). */
double orc_holecut(int ngrids, const int32_t *dims, const double *const *X, const double *const *Y,
                   const double *const *Z, const int32_t *blank_kind, const double *blank_prm,
                   const double *poses, const int64_t *node_off, uint8_t *flags, const double *const *mesh_tri,
                   const int64_t *mesh_ntri) {
    double min_gap = INFINITY;
    double *mbox = (double *)malloc(sizeof(double) * 6 * (size_t)ngrids);
    for (int B = 0; B < ngrids; ++B)
        if (blank_kind[B] == BLANK_MESH) mesh_box(mesh_tri[B], mesh_ntri[B], mbox + 6 * B);
    for (int A = 0; A < ngrids; ++A) {
        int64_t n = (int64_t)dims[4 * A] * dims[4 * A + 1] * dims[4 * A + 2];
        const double *pa = poses + 12 * A;
        double gmin = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : gmin)
        for (int64_t m = 0; m < n; ++m) {
            double w[3];
            apply_pose(pa, X[A][m], Y[A][m], Z[A][m], w);
            uint8_t f = ST_FIELD;
            for (int B = 0; B < ngrids; ++B) {
                if (B == A || blank_kind[B] == BLANK_NONE) continue;
                double xi[3], gap;
                apply_pose_inv(poses + 12 * B, w, xi);
                int in = blank_kind[B] == BLANK_MESH
                             ? mesh_inside(mesh_tri[B], mesh_ntri[B], mbox + 6 * B, xi, &gap)
                             : blank_inside(blank_kind[B], blank_prm + 8 * B, xi, &gap);
                if (gap < gmin) gmin = gap;
                if (in) {
                    f = (uint8_t)(ST_HOLE | (B << 2));
                    break;
                }
            }
            flags[node_off[A] + m] = f;
        }
        if (gmin < min_gap) min_gap = gmin;
    }
    free(mbox);
    return min_gap;
}

/* ------------------------------------------------------------ fringe */
static int wrap_index(int v, int n, int periodic) {
    if (periodic) {
        v %= n;
        if (v < 0) v += n;
        return v;
    }
    return (v < 0 || v >= n) ? -1 : v;
}

/* outer: [ngrids*6] layers on faces i-, i+, j-, j+, k-, k+. */
void orc_fringe(int ngrids, const int32_t *dims, const int32_t *outer, int nf,
                const int64_t *node_off, uint8_t *flags) {
    for (int A = 0; A < ngrids; ++A) {
        int ni = dims[4 * A], nj = dims[4 * A + 1], nk = dims[4 * A + 2], per = dims[4 * A + 3];
        int64_t n = (int64_t)ni * nj * nk;
        uint8_t *fl = flags + node_off[A];
        const int32_t *o = outer + 6 * A;
        uint8_t *cause = (uint8_t *)malloc((size_t)n);
        /* overset boundary faces: potential query points (Sec. 2.2.3, item 1) */
        for (int64_t m = 0; m < n; ++m) {
            int i = (int)(m % ni), j = (int)((m / ni) % nj), k = (int)(m / ((int64_t)ni * nj));
            int onb = i < o[0] || i >= ni - o[1] || j < o[2] || j >= nj - o[3] || k < o[4] || k >= nk - o[5];
            cause[m] = onb ? CAUSE_BOUNDARY : 255;
        }
        /* buffer layer: every non-hole node within Chebyshev distance nf of a hole */
        for (int64_t m = 0; m < n; ++m) {
            if ((fl[m] & 3) != ST_HOLE) continue;
            uint8_t hc = (uint8_t)(fl[m] >> 2);
            int i = (int)(m % ni), j = (int)((m / ni) % nj), k = (int)(m / ((int64_t)ni * nj));
            for (int dk = -nf; dk <= nf; ++dk) {
                int kk = wrap_index(k + dk, nk, per & 4);
                if (kk < 0) continue;
                for (int dj = -nf; dj <= nf; ++dj) {
                    int jj = wrap_index(j + dj, nj, per & 2);
                    if (jj < 0) continue;
                    for (int di = -nf; di <= nf; ++di) {
                        int ii = wrap_index(i + di, ni, per & 1);
                        if (ii < 0) continue;
                        int64_t q = ii + (int64_t)ni * (jj + (int64_t)nj * kk);
                        if ((fl[q] & 3) == ST_HOLE) continue;
                        if (hc < cause[q]) cause[q] = hc;
                    }
                }
            }
        }
        for (int64_t m = 0; m < n; ++m) {
            if ((fl[m] & 3) == ST_HOLE) continue;
            fl[m] = cause[m] == 255 ? (uint8_t)ST_FIELD : (uint8_t)(ST_FRINGE | (cause[m] << 2));
        }
        free(cause);
    }
}

/* ------------------------------------------------------------ compaction */
/* Fringe nodes in ascending (grid, linear node) order. Writes at most
 * `capacity` entries; returns the total count. */
int64_t orc_compact(int ngrids, const int64_t *node_off, const uint8_t *flags,
                    int32_t *q_grid, int32_t *q_node, int64_t capacity) {
    int64_t cnt = 0;
    for (int A = 0; A < ngrids; ++A) {
        for (int64_t m = node_off[A]; m < node_off[A + 1]; ++m) {
            if ((flags[m] & 3) != ST_FRINGE) continue;
            if (cnt < capacity) {
                q_grid[cnt] = A;
                q_node[cnt] = (int32_t)(m - node_off[A]);
            }
            ++cnt;
        }
    }
    return cnt;
}

/* ------------------------------------------------------------ cells */
typedef struct {
    int ni, nj, nk, per, nci, ncj, nck;
} gdim;

static gdim make_dim(const int32_t *d) {
    gdim g;
    g.ni = d[0]; g.nj = d[1]; g.nk = d[2]; g.per = d[3];
    g.nci = (g.per & 1) ? g.ni : g.ni - 1;
    g.ncj = (g.per & 2) ? g.nj : g.nj - 1;
    g.nck = (g.per & 4) ? g.nk : g.nk - 1;
    return g;
}

/* Node indices of the 8 corners of a cell, corner c = c0 + 2 c1 + 4 c2 with
 * c0 the i offset (fastest); periodic directions wrap. */
static void cell_corners(const gdim *g, int64_t cell, int64_t nodes[8]) {
    int ci = (int)(cell % g->nci);
    int cj = (int)((cell / g->nci) % g->ncj);
    int ck = (int)(cell / ((int64_t)g->nci * g->ncj));
    for (int c = 0; c < 8; ++c) {
        int i = ci + (c & 1), j = cj + ((c >> 1) & 1), k = ck + ((c >> 2) & 1);
        if (i == g->ni) i = 0;
        if (j == g->nj) j = 0;
        if (k == g->nk) k = 0;
        nodes[c] = i + (int64_t)g->ni * (j + (int64_t)g->nj * k);
    }
}

/* ------------------------------------------------------------ control cells */
typedef struct {
    double lo[3], inv[3];
    int nb[3];
    int64_t *start;   /* [nbins + 1] */
    int32_t *cells;   /* candidate donor cells of each control cell (any order) */
} orc_bins;

static void cell_aabb(const gdim *g, const double *X, const double *Y, const double *Z,
                      int64_t cell, double lo[3], double hi[3]) {
    int64_t nd[8];
    cell_corners(g, cell, nd);
    lo[0] = hi[0] = X[nd[0]];
    lo[1] = hi[1] = Y[nd[0]];
    lo[2] = hi[2] = Z[nd[0]];
    for (int c = 1; c < 8; ++c) {
        double v[3] = {X[nd[c]], Y[nd[c]], Z[nd[c]]};
        for (int d = 0; d < 3; ++d) {
            if (v[d] < lo[d]) lo[d] = v[d];
            if (v[d] > hi[d]) hi[d] = v[d];
        }
    }
    /* pad far beyond the containment tolerance so that no containing cell is lost */
    double ext = hi[0] - lo[0];
    if (hi[1] - lo[1] > ext) ext = hi[1] - lo[1];
    if (hi[2] - lo[2] > ext) ext = hi[2] - lo[2];
    double pad = 1e-9 * ext + 1e-300;
    for (int d = 0; d < 3; ++d) {
        lo[d] -= pad;
        hi[d] += pad;
    }
}

static int bin_coord(const orc_bins *b, int d, double v) {
    double t = (v - b->lo[d]) * b->inv[d];
    int i = (int)floor(t);
    if (i < 0) i = 0;
    if (i >= b->nb[d]) i = b->nb[d] - 1;
    return i;
}

/* Control cells over the grid's axis-aligned bounding box (body frame): about
 * one control cell per 8 donor cells, shaped after the box. A donor cell is
 * listed in every control cell its padded corner box overlaps, so any point
 * inside a donor cell finds that cell in the list of its control cell. */
orc_bins *orc_bins_build(const int32_t *dims, const double *X, const double *Y, const double *Z) {
    gdim g = make_dim(dims);
    int64_t ncell = (int64_t)g.nci * g.ncj * g.nck;
    int64_t nn = (int64_t)g.ni * g.nj * g.nk;
    orc_bins *b = (orc_bins *)calloc(1, sizeof(orc_bins));
    double lo[3] = {X[0], Y[0], Z[0]}, hi[3] = {X[0], Y[0], Z[0]};
    for (int64_t m = 0; m < nn; ++m) {
        double v[3] = {X[m], Y[m], Z[m]};
        for (int d = 0; d < 3; ++d) {
            if (v[d] < lo[d]) lo[d] = v[d];
            if (v[d] > hi[d]) hi[d] = v[d];
        }
    }
    double ext[3], gm = 1.0;
    for (int d = 0; d < 3; ++d) {
        ext[d] = hi[d] - lo[d];
        if (ext[d] <= 0) ext[d] = 1e-30;
        gm *= ext[d];
    }
    gm = cbrt(gm);
    double per_axis = cbrt((double)ncell / 8.0);
    for (int d = 0; d < 3; ++d) {
        int nb = (int)ceil(per_axis * ext[d] / gm);
        if (nb < 1) nb = 1;
        if (nb > 2048) nb = 2048;
        b->nb[d] = nb;
        b->lo[d] = lo[d];
        b->inv[d] = nb / ext[d];
    }
    int64_t nbins = (int64_t)b->nb[0] * b->nb[1] * b->nb[2];
    b->start = (int64_t *)calloc((size_t)nbins + 1, sizeof(int64_t));
    int64_t *cursor = NULL;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int64_t q = 0; q < nbins; ++q) b->start[q + 1] += b->start[q];
            b->cells = (int32_t *)malloc(sizeof(int32_t) * (size_t)(b->start[nbins] > 0 ? b->start[nbins] : 1));
            cursor = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nbins > 0 ? nbins : 1));
            memcpy(cursor, b->start, sizeof(int64_t) * (size_t)nbins);
        }
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < ncell; ++c) {
            double clo[3], chi[3];
            cell_aabb(&g, X, Y, Z, c, clo, chi);
            int a0 = bin_coord(b, 0, clo[0]), a1 = bin_coord(b, 0, chi[0]);
            int b0 = bin_coord(b, 1, clo[1]), b1 = bin_coord(b, 1, chi[1]);
            int e0 = bin_coord(b, 2, clo[2]), e1 = bin_coord(b, 2, chi[2]);
            for (int z = e0; z <= e1; ++z)
                for (int y = b0; y <= b1; ++y)
                    for (int x = a0; x <= a1; ++x) {
                        int64_t q = x + (int64_t)b->nb[0] * (y + (int64_t)b->nb[1] * z);
                        if (pass == 0) {
#pragma omp atomic
                            b->start[q + 1]++;
                        } else {
                            int64_t slot;
#pragma omp atomic capture
                            slot = cursor[q]++;
                            b->cells[slot] = (int32_t)c;
                        }
                    }
        }
    }
    free(cursor);
    return b;
}

void orc_bins_free(orc_bins *b) {
    if (!b) return;
    free(b->start);
    free(b->cells);
    free(b);
}

int64_t orc_bins_entries(const orc_bins *b) {
    return b->start[(int64_t)b->nb[0] * b->nb[1] * b->nb[2]];
}

/* ------------------------------------------------------------ Newton */
/* Solve J d = r by Gaussian elimination with partial pivoting; 0 if singular. */
static int solve3(double J[3][3], double r[3], double d[3]) {
    double a[3][4];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) a[i][j] = J[i][j];
        a[i][3] = r[i];
    }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int i = col + 1; i < 3; ++i)
            if (fabs(a[i][col]) > fabs(a[piv][col])) piv = i;
        if (a[piv][col] == 0.0) return 0;
        if (piv != col)
            for (int j = 0; j < 4; ++j) {
                double t = a[col][j];
                a[col][j] = a[piv][j];
                a[piv][j] = t;
            }
        for (int i = col + 1; i < 3; ++i) {
            double f = a[i][col] / a[col][col];
            for (int j = col; j < 4; ++j) a[i][j] = a[i][j] - f * a[col][j];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double v = a[i][3];
        for (int j = i + 1; j < 3; ++j) v = v - a[i][j] * d[j];
        d[i] = v / a[i][i];
    }
    return 1;
}

/* Trilinear map of the cell, x(s) = sum_c N_c(s) P_c, N_c = prod_d (c_d ? s_d : 1 - s_d),
 * and its Jacobian dx/ds. */
static void trilinear_eval(const double P[8][3], const double s[3], double x[3], double J[3][3]) {
    for (int i = 0; i < 3; ++i) {
        x[i] = 0.0;
        J[i][0] = J[i][1] = J[i][2] = 0.0;
    }
    for (int c = 0; c < 8; ++c) {
        double f[3], df[3];
        for (int d = 0; d < 3; ++d) {
            int bit = (c >> d) & 1;
            f[d] = bit ? s[d] : 1.0 - s[d];
            df[d] = bit ? 1.0 : -1.0;
        }
        double N = (f[0] * f[1]) * f[2];
        double dN[3] = {(df[0] * f[1]) * f[2], (f[0] * df[1]) * f[2], (f[0] * f[1]) * df[2]};
        for (int i = 0; i < 3; ++i) {
            x[i] = x[i] + N * P[c][i];
            for (int d = 0; d < 3; ++d) J[i][d] = J[i][d] + dN[d] * P[c][i];
        }
    }
}

/* Natural coordinates of xi in the cell by Newton's method from s = (1/2,1/2,1/2).
 * Returns 1 if converged (last step <= NEWTON_TOL, final |det J| >= DET_MIN). */
static int newton_natural(const double P[8][3], const double xi[3], double s[3]) {
    s[0] = s[1] = s[2] = 0.5;
    for (int it = 0; it < NEWTON_MAXIT; ++it) {
        double x[3], J[3][3], r[3], d[3];
        trilinear_eval(P, s, x, J);
        for (int i = 0; i < 3; ++i) r[i] = x[i] - xi[i];
        if (!solve3(J, r, d)) return 0;
        double dmax = 0.0;
        for (int i = 0; i < 3; ++i) {
            s[i] = s[i] - d[i];
            if (fabs(d[i]) > dmax) dmax = fabs(d[i]);
        }
        if (!(dmax == dmax)) return 0; /* NaN */
        if (dmax <= NEWTON_TOL) {
            trilinear_eval(P, s, x, J);
            double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            return fabs(det) >= DET_MIN;
        }
    }
    return 0;
}

/* Try one candidate cell: 1 if xi lies in it (natural coordinates in the
 * closed unit cube up to S_TOL); s receives the coordinates. */
static int cell_contains(const gdim *g, const double *X, const double *Y, const double *Z,
                         int64_t cell, const double xi[3], double s[3]) {
    int64_t nd[8];
    double P[8][3];
    cell_corners(g, cell, nd);
    for (int c = 0; c < 8; ++c) {
        P[c][0] = X[nd[c]];
        P[c][1] = Y[nd[c]];
        P[c][2] = Z[nd[c]];
    }
    if (!newton_natural(P, xi, s)) return 0;
    for (int d = 0; d < 3; ++d)
        if (s[d] < -S_TOL || s[d] > 1.0 + S_TOL) return 0;
    return 1;
}

static int cell_valid(const gdim *g, int64_t cell, const uint8_t *fl) {
    int64_t nd[8];
    cell_corners(g, cell, nd);
    for (int c = 0; c < 8; ++c)
        if ((fl[nd[c]] & 3) == ST_HOLE) return 0;
    return 1;
}

static int point_in_box(const double lo[3], const double hi[3], const double p[3]) {
    return p[0] >= lo[0] && p[0] <= hi[0] && p[1] >= lo[1] && p[1] <= hi[1] && p[2] >= lo[2] && p[2] <= hi[2];
}

/* Candidate donor grids of a query of grid A whose flag carries `cause`:
 * the cause grid, then the background (grid 0), then ascending ids (Sec. 2.4, item 1). */
static int candidate_grids(int ngrids, int A, int cause, int out[64]) {
    int n = 0;
    if (cause != CAUSE_BOUNDARY && cause != A && cause < ngrids) out[n++] = cause;
    if (A != 0 && !(n == 1 && out[0] == 0)) out[n++] = 0;
    for (int g = 0; g < ngrids; ++g) {
        int dup = (g == A);
        for (int t = 0; t < n; ++t) dup |= (out[t] == g);
        if (!dup) out[n++] = g;
    }
    return n;
}

/* Donor search (Sec. 2.2.5) for nq queries (q_grid, q_node).
 * bins: one control-cell structure per grid (ignored when exhaustive != 0,
 * in which case every cell of every candidate grid is tried: the plain
 * definition, for tiny grids). Outputs: donor grid and cell (-1 for orphans),
 * s (3 per query, NaN for orphans), margin min_d min(s_d, 1 - s_d). */
void orc_donor_search(int ngrids, const int32_t *dims, const double *const *X, const double *const *Y,
                      const double *const *Z, const int64_t *node_off, const uint8_t *flags,
                      const double *poses, orc_bins *const *bins, int exhaustive, int64_t nq,
                      const int32_t *q_grid, const int32_t *q_node, int32_t *donor_grid,
                      int32_t *donor_cell, double *s_out, double *margin) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nq; ++q) {
        int A = q_grid[q];
        int64_t m = q_node[q];
        double w[3];
        apply_pose(poses + 12 * A, X[A][m], Y[A][m], Z[A][m], w);
        int cause = flags[node_off[A] + m] >> 2;
        int cand[64];
        int nc = candidate_grids(ngrids, A, cause, cand);
        donor_grid[q] = -1;
        donor_cell[q] = -1;
        s_out[3 * q] = s_out[3 * q + 1] = s_out[3 * q + 2] = NAN;
        margin[q] = NAN;
        for (int t = 0; t < nc; ++t) {
            int B = cand[t];
            gdim g = make_dim(dims + 4 * B);
            const uint8_t *fl = flags + node_off[B];
            double xi[3];
            apply_pose_inv(poses + 12 * B, w, xi);
            int64_t best = -1;
            double sb[3] = {0, 0, 0};
            int64_t ncell = (int64_t)g.nci * g.ncj * g.nck;
            int64_t c0 = 0, c1 = ncell;
            const int32_t *list = NULL;
            if (!exhaustive) {
                const orc_bins *b = bins[B];
                double lo[3] = {b->lo[0], b->lo[1], b->lo[2]};
                double hi[3] = {b->lo[0] + b->nb[0] / b->inv[0], b->lo[1] + b->nb[1] / b->inv[1],
                                b->lo[2] + b->nb[2] / b->inv[2]};
                /* points outside the control-cell box lie in no cell (boxes are padded) */
                double pad = 1e-6 * ((hi[0] - lo[0]) + (hi[1] - lo[1]) + (hi[2] - lo[2]));
                for (int d = 0; d < 3; ++d) {
                    lo[d] -= pad;
                    hi[d] += pad;
                }
                if (!point_in_box(lo, hi, xi)) continue;
                int64_t bq = bin_coord(b, 0, xi[0]) +
                             (int64_t)b->nb[0] * (bin_coord(b, 1, xi[1]) + (int64_t)b->nb[1] * bin_coord(b, 2, xi[2]));
                c0 = b->start[bq];
                c1 = b->start[bq + 1];
                list = b->cells;
            }
            for (int64_t e = c0; e < c1; ++e) {
                int64_t cell = list ? list[e] : e;
                if (best >= 0 && cell >= best) continue;
                if (list) {
                    double lo[3], hi[3];
                    cell_aabb(&g, X[B], Y[B], Z[B], cell, lo, hi);
                    if (!point_in_box(lo, hi, xi)) continue;
                }
                double s[3];
                if (!cell_contains(&g, X[B], Y[B], Z[B], cell, xi, s)) continue;
                if (!cell_valid(&g, cell, fl)) continue;
                best = cell;
                sb[0] = s[0];
                sb[1] = s[1];
                sb[2] = s[2];
            }
            if (best >= 0) {
                donor_grid[q] = B;
                donor_cell[q] = (int32_t)best;
                double mg = 1.0;
                for (int d = 0; d < 3; ++d) {
                    s_out[3 * q + d] = sb[d];
                    double a = sb[d] < 1.0 - sb[d] ? sb[d] : 1.0 - sb[d];
                    if (a < mg) mg = a;
                }
                margin[q] = mg;
                break;
            }
        }
    }
}

/* Natural coordinates of xi in one given cell (diagnostics: validity of a
 * donor chosen elsewhere). Returns 1 if Newton converged. */
int orc_cell_coords(const int32_t *dims, const double *X, const double *Y, const double *Z,
                    int64_t cell, const double *xi, double *s) {
    gdim g = make_dim(dims);
    int64_t nd[8];
    double P[8][3];
    cell_corners(&g, cell, nd);
    for (int c = 0; c < 8; ++c) {
        P[c][0] = X[nd[c]];
        P[c][1] = Y[nd[c]];
        P[c][2] = Z[nd[c]];
    }
    return newton_natural(P, xi, s);
}

/* ------------------------------------------------------------ interpolation */
/* q_p = sum_{c=0..7} w_c q_c, w_c = prod_d (c_d ? s_d : 1 - s_d), summed in
 * ascending c (Sec. 2.2.6). fields: [nfields][total nodes]; out: [nfields][nq].
 * Orphans (donor_grid < 0) are left untouched. */
void orc_interp(int ngrids, const int32_t *dims, const int64_t *node_off, int64_t total_nodes,
                int nfields, const double *fields, int64_t nq, const int32_t *donor_grid,
                const int32_t *donor_cell, const double *s, double *out) {
    (void)ngrids;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nq; ++q) {
        int B = donor_grid[q];
        if (B < 0) continue;
        gdim g = make_dim(dims + 4 * B);
        int64_t nd[8];
        cell_corners(&g, donor_cell[q], nd);
        double wgt[8];
        for (int c = 0; c < 8; ++c) {
            double f[3];
            for (int d = 0; d < 3; ++d) f[d] = ((c >> d) & 1) ? s[3 * q + d] : 1.0 - s[3 * q + d];
            wgt[c] = (f[0] * f[1]) * f[2];
        }
        for (int fld = 0; fld < nfields; ++fld) {
            const double *F = fields + (int64_t)fld * total_nodes + node_off[B];
            double acc = 0.0;
            for (int c = 0; c < 8; ++c) acc = acc + wgt[c] * F[nd[c]];
            out[(int64_t)fld * nq + q] = acc;
        }
    }
}

/* Weights alone (for invariant checks). */
void orc_weights(const double *s, double *w) {
    for (int c = 0; c < 8; ++c) {
        double f[3];
        for (int d = 0; d < 3; ++d) f[d] = ((c >> d) & 1) ? s[d] : 1.0 - s[d];
        w[c] = (f[0] * f[1]) * f[2];
    }
}

/* Velocity in the receiver's frame (Sec. 2.3): the fields interpolated from
 * donor grid B are components in B's non-inertial frame; the receiver, a
 * node of grid A, needs them in A's frame. With poses x = R X + c (R = Q^T of
 * the paper), the inertial velocity is R_B u_B and A's components are
 * u_A = R_A^T (R_B u_B). Fields 0, 1, 2 of values (nfields blocks of nq) are
 * rewritten in place; queries without a donor are left alone. */
void orc_frame_velocity(const double *poses, int64_t nq, const int32_t *q_grid, const int32_t *donor_grid,
                        double *values) {
    for (int64_t q = 0; q < nq; ++q) {
        int B = donor_grid[q];
        if (B < 0) continue;
        const double *rb = poses + 12 * B, *ra = poses + 12 * q_grid[q];
        double u[3] = {values[q], values[nq + q], values[2 * nq + q]}, w[3];
        for (int i = 0; i < 3; ++i) w[i] = (rb[3 * i] * u[0] + rb[3 * i + 1] * u[1]) + rb[3 * i + 2] * u[2];
        for (int i = 0; i < 3; ++i) values[i * nq + q] = (ra[i] * w[0] + ra[3 + i] * w[1]) + ra[6 + i] * w[2];
    }
}

/* The interpolation matrix (Sec. 2.2.6, second option; Alg. 4): row q
 * holds, for its 8 corners c, the global index of the corner node (grids
 * packed by node offset, the paper's global index with one process) and
 * the trilinear weight w_c = prod_d (c_d ? s_d : 1 - s_d). A query without a
 * donor has an empty row: index -1, weight 0. */
void orc_interp_matrix(const int32_t *dims, const int64_t *node_off, int64_t nq, const int32_t *donor_grid,
                       const int32_t *donor_cell, const double *s, int64_t *cols, double *vals) {
    for (int64_t q = 0; q < nq; ++q) {
        int B = donor_grid[q];
        if (B < 0) {
            for (int c = 0; c < 8; ++c) {
                cols[8 * q + c] = -1;
                vals[8 * q + c] = 0.0;
            }
            continue;
        }
        gdim g = make_dim(dims + 4 * B);
        int64_t nd[8];
        cell_corners(&g, donor_cell[q], nd);
        for (int c = 0; c < 8; ++c) {
            double f[3];
            for (int d = 0; d < 3; ++d) f[d] = ((c >> d) & 1) ? s[3 * q + d] : 1.0 - s[3 * q + d];
            cols[8 * q + c] = node_off[B] + nd[c];
            vals[8 * q + c] = (f[0] * f[1]) * f[2];
        }
    }
}

/* y_r = M x_r for nrhs vectors x_r (blocks of total_nodes), y as nrhs
 * blocks of nq. Empty entries (index -1) contribute nothing. */
void orc_matrix_apply(int64_t nq, const int64_t *cols, const double *vals, int nrhs, int64_t total_nodes,
                      const double *x, double *y) {
    for (int r = 0; r < nrhs; ++r)
        for (int64_t q = 0; q < nq; ++q) {
            double acc = 0.0;
            for (int c = 0; c < 8; ++c) {
                int64_t j = cols[8 * q + c];
                if (j >= 0) acc = acc + vals[8 * q + c] * x[(int64_t)r * total_nodes + j];
            }
            y[(int64_t)r * nq + q] = acc;
        }
}
