// Donor search on gfx950 (Sec. 2.2.5 and Alg. 3 of arXiv:1910.09315, donor
// selection of Sec. 2.4 item 1).
//
// One query per lane. For each candidate donor grid the query is taken into
// that grid's body frame (in FP64), then a stencil walk moves from a seed cell
// (last step's donor, else the lowest cell of the query's control cell)
// toward the cell whose trilinear natural coordinates s, found by Newton's
// method, lie in [0,1]^3. Alg. 3 steps by the signs of face distances; here
// the signs of s and s-1 play that role (their sign pattern is what the
// face tests measure, and Newton's s is needed for containment anyway).
// A walk that leaves the grid, revisits its previous cell, meets a blanked
// donor or runs out of steps hands over to the brute-force scan of the
// control cell (Alg. 3, label nxtp), which keeps the lowest valid containing
// cell index. The walk only accelerates: the scan defines the result.
//
// Precision: the natural-coordinate solve runs in T. With T = float (mixed
// precision) every offset is formed in FP64 from FP64 corners and only then
// rounded, so the FP32 solve sees cell-local quantities. The query position
// of an overset node comes from the FP32 transform and carries its rounding
// error e (bounded per component from |qx|); a result is kept only if its
// FP32 margin to every face is >= 1e-4 plus that error carried into natural
// coordinates (2 sqrt(3) e ||J^-1||_F) and the cell's Jacobian condition
// estimate is <= 1e3. Otherwise the walk continues in FP64 from that cell
// (the FP64 correction), on the position recomputed in FP64 from the FP64
// node coordinates; the brute-force scans also use that exact position.
#include <hip/hip_runtime.h>

#include "ov_internal.h"

namespace ov {

constexpr float kMixedMargin = 1e-4f;
constexpr float kMixedCond = 1e3f;
// FP32 steps on only when the point is at least this far outside the cell
// (in natural coordinates); nearer, FP64 takes over.
constexpr float kClearlyOutside = 1e-2f;
constexpr float kNewtonTolF = 2e-6f;
constexpr int kNewtonMaxItF = 16;

enum WalkResult { kFound = 1, kToScan = 0, kDoubt = 2 };

// Trilinear map of a cell relative to its corner 0:
//   x(s) - P0 = a1 s0 + a2 s1 + a3 s2 + a4 s0 s1 + a5 s0 s2 + a6 s1 s2 + a7 s0 s1 s2,
// coefficients formed in FP64 from the corners and rounded to T.
template <typename T>
struct CellMap {
  T a[8][3];  // a[1..7]
  T e[3];     // query - P0
};

template <typename T>
__device__ __forceinline__ void map_from_corners(const double P[8][3], const double xi[3], CellMap<T>& m) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double p0 = P[0][d];
    double q1 = P[1][d] - p0, q2 = P[2][d] - p0, q3 = P[3][d] - p0, q4 = P[4][d] - p0;
    double q5 = P[5][d] - p0, q6 = P[6][d] - p0, q7 = P[7][d] - p0;
    m.e[d] = (T)(xi[d] - p0);
    m.a[1][d] = (T)q1;
    m.a[2][d] = (T)q2;
    m.a[3][d] = (T)q4;
    m.a[4][d] = (T)(q3 - q1 - q2);
    m.a[5][d] = (T)(q5 - q1 - q4);
    m.a[6][d] = (T)(q6 - q2 - q4);
    m.a[7][d] = (T)(q7 - q3 - q5 - q6 + q1 + q2 + q4);
  }
}

template <typename T>
__device__ __forceinline__ void load_cell(const GridDev& G, int ci, int cj, int ck, const double xi[3],
                                          CellMap<T>& m) {
  if (sizeof(T) == 4 && G.PF) {
    // the FP32 walk: corners from the FP32 layout (16 bytes each, offsets
    // from the grid's anchor); the query's offset from corner 0 formed in
    // FP64 and then rounded. The corners' rounding (pf_err per component)
    // enters the walk's acceptance test.
    float P[8][3];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const ov_fv4 v = ((gmem<ov_fv4>*)gp((const float*)G.PF))[corner_node(G, ci, cj, ck, c)];
      P[c][0] = v.x;
      P[c][1] = v.y;
      P[c][2] = v.z;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float p0 = P[0][d];
      const float q1 = P[1][d] - p0, q2 = P[2][d] - p0, q3 = P[3][d] - p0, q4 = P[4][d] - p0;
      const float q5 = P[5][d] - p0, q6 = P[6][d] - p0, q7 = P[7][d] - p0;
      m.e[d] = (T)((xi[d] - G.anchor[d]) - (double)p0);
      m.a[1][d] = (T)q1;
      m.a[2][d] = (T)q2;
      m.a[3][d] = (T)q4;
      m.a[4][d] = (T)(q3 - q1 - q2);
      m.a[5][d] = (T)(q5 - q1 - q4);
      m.a[6][d] = (T)(q6 - q2 - q4);
      m.a[7][d] = (T)(q7 - q3 - q5 - q6 + q1 + q2 + q4);
    }
    return;
  }
  double P[8][3];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    load_xyz(G, corner_node(G, ci, cj, ck, c), P[c][0], P[c][1], P[c][2]);
  }
  map_from_corners<T>(P, xi, m);
}

template <typename T>
__device__ __forceinline__ void map_and_jacobian(const CellMap<T>& m, const T s[3], T r[3], T J[3][3]) {
  T st = s[0] * s[1], su = s[0] * s[2], tu = s[1] * s[2], stu = st * s[2];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    r[d] = m.a[1][d] * s[0] + m.a[2][d] * s[1] + m.a[3][d] * s[2] + m.a[4][d] * st + m.a[5][d] * su +
           m.a[6][d] * tu + m.a[7][d] * stu - m.e[d];
    J[d][0] = m.a[1][d] + m.a[4][d] * s[1] + m.a[5][d] * s[2] + m.a[7][d] * tu;
    J[d][1] = m.a[2][d] + m.a[4][d] * s[0] + m.a[6][d] * s[2] + m.a[7][d] * su;
    J[d][2] = m.a[3][d] + m.a[5][d] * s[0] + m.a[6][d] * s[1] + m.a[7][d] * st;
  }
}

// 1 / x for Newton's update: the hardware reciprocal (FP32: within 1 ulp),
// in FP64 refined by two Newton-Raphson steps r <- r + r (1 - x r), each of
// which squares the relative error. Newton's iteration needs no correctly
// rounded quotient, and this is a shorter dependent chain than a division.
template <typename T>
__device__ __forceinline__ T recip(T x);
template <>
__device__ __forceinline__ float recip<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ __forceinline__ double recip<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}

template <typename T>
__device__ __forceinline__ T det3(const T J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Newton's method for x(s) = query from the s given (the cell's centre, or a
// point carried over from a neighbouring cell). Returns true when the last
// step is <= tol (and, in FP64, |det J| >= kDetMin at the result).
// *cond receives ||J||_F ||J^-1||_F at the result (an upper bound of the
// 2-norm condition number).
// *inv_norm receives ||J^-1||_F at the result.
// *iters (if given) is increased by the iterations taken.
template <typename T>
__device__ bool newton(const CellMap<T>& m, T s[3], T* cond, T* inv_norm = nullptr, int* iters = nullptr) {
  const T tol = sizeof(T) == 8 ? (T)kNewtonTol : (T)kNewtonTolF;
  const int maxit = sizeof(T) == 8 ? kNewtonMaxIt : kNewtonMaxItF;
  for (int it = 0; it < maxit; ++it) {
    if (iters) ++*iters;
    T r[3], J[3][3];
    map_and_jacobian(m, s, r, J);
    // Cramer's rule with the columns of J
    T c12[3] = {J[1][1] * J[2][2] - J[2][1] * J[1][2], J[2][1] * J[0][2] - J[0][1] * J[2][2],
                J[0][1] * J[1][2] - J[1][1] * J[0][2]};
    T det = J[0][0] * c12[0] + J[1][0] * c12[1] + J[2][0] * c12[2];
    if (det == (T)0) return false;
    const T inv = recip<T>(det);
    T d0 = (r[0] * c12[0] + r[1] * c12[1] + r[2] * c12[2]) * inv;
    // column 1 replaced by r: det[J0, r, J2] = J0 . (r x J2)
    T rx2[3] = {r[1] * J[2][2] - r[2] * J[1][2], r[2] * J[0][2] - r[0] * J[2][2], r[0] * J[1][2] - r[1] * J[0][2]};
    T d1 = (J[0][0] * rx2[0] + J[1][0] * rx2[1] + J[2][0] * rx2[2]) * inv;
    // column 2 replaced by r: det[J0, J1, r] = J0 . (J1 x r)
    T j1r[3] = {J[1][1] * r[2] - J[2][1] * r[1], J[2][1] * r[0] - J[0][1] * r[2], J[0][1] * r[1] - J[1][1] * r[0]};
    T d2 = (J[0][0] * j1r[0] + J[1][0] * j1r[1] + J[2][0] * j1r[2]) * inv;
    s[0] -= d0;
    s[1] -= d1;
    s[2] -= d2;
    T dm = fmax(fabs(d0), fmax(fabs(d1), fabs(d2)));
    if (!(dm == dm) || !(fabs(s[0]) < (T)1e6 && fabs(s[1]) < (T)1e6 && fabs(s[2]) < (T)1e6)) return false;
    if (dm <= tol) {
      map_and_jacobian(m, s, r, J);
      T dt = det3(J);
      if (sizeof(T) == 8 && !(fabs((double)dt) >= kDetMin)) return false;
      if (dt == (T)0) return false;
      if (cond) {
        T nj = 0, na = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            nj += J[i][j] * J[i][j];
            // cofactor (i, j)
            int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            T cf = J[i1][j1] * J[i2][j2] - J[i1][j2] * J[i2][j1];
            na += cf * cf;
          }
        const T in = sqrt(na) * recip<T>(fabs(dt));
        *cond = sqrt(nj) * in;
        if (inv_norm) *inv_norm = in;
      }
      return true;
    }
  }
  return false;
}

// Newton's start in the first cell of a walk: a point of [0, 1]^3, or (on =
// false) the cell's centre. Passed by value, so that it stays in registers.
struct Start {
  double v[3];
  bool on;
};
constexpr Start kCentre = {{0.5, 0.5, 0.5}, false};

// A start from a solve's result: each component clamped to [0, 1] (a NaN
// component, as a failed solve leaves, becomes 1/2).
template <typename T>
__device__ __forceinline__ Start start_from(const T s[3]) {
  Start r;
  r.on = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double v = (double)s[d];
    r.v[d] = v == v ? fmin(fmax(v, 0.0), 1.0) : 0.5;
  }
  return r;
}

template <typename T>
__device__ __forceinline__ bool inside(const T s[3], T tol) {
  return s[0] >= -tol && s[0] <= (T)1 + tol && s[1] >= -tol && s[1] <= (T)1 + tol && s[2] >= -tol &&
         s[2] <= (T)1 + tol;
}

__device__ __forceinline__ bool cell_valid(const GridDev& G, const uint8_t* fl, int ci, int cj, int ck) {
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 8; ++c) ok &= (fl[corner_node(G, ci, cj, ck, c)] & 3) != kHole;
  return ok;
}

// Whether a tile holding a corner of the cell holds a hole this step, from
// the step's map of tiles holding a hole (a few bytes that stay in cache):
// a cell none of whose tiles does is valid without reading its 8 flag bytes
// (each on its own line). th: the map of the step's slot (null: true, the
// flags decide).
__device__ __forceinline__ bool corner_tiles_hold_hole(const GridDev& G, int ci, int cj, int ck,
                                                       const unsigned int* th, unsigned int stamp) {
  if (!th) return true;
  bool hole_tile = false;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    int i = ci + (c & 1), j = cj + ((c >> 1) & 1), k = ck + ((c >> 2) & 1);
    i = (i == G.ni) ? 0 : i;
    j = (j == G.nj) ? 0 : j;
    k = (k == G.nk) ? 0 : k;
    hole_tile |= gp(th)[G.tile_off + (i >> 6) + (long long)G.tiles_i * ((j >> 3) + (long long)G.tiles_j * (k >> 3))] ==
                 stamp;
  }
  return hole_tile;
}

// The same test on flags already loaded (the walk fetches a cell's corner
// flags together with its corner coordinates: one memory round trip).
__device__ __forceinline__ bool corners_valid(const uint8_t cf[8]) {
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 8; ++c) ok &= (cf[c] & 3) != kHole;
  return ok;
}

// One axis of a walk step. A periodic step is at most max(2, nc / 4)
// cells from a cell in [0, nc) (nc >= 2), so one wrap brings it back.
__device__ __forceinline__ int step_axis(int v, int dv, int nc, bool periodic, bool& clamped) {
  int w = v + dv;
  if (periodic) {
    if (w < 0) w += nc;
    else if (w >= nc) w -= nc;
    return w;
  }
  if (w < 0) {
    clamped = true;
    return 0;
  }
  if (w >= nc) {
    clamped = true;
    return nc - 1;
  }
  return w;
}

// One axis of a walk step that went past a polar end (GridDev::pole; ends:
// bit 0 low, bit 1 high): the step goes on in the cells across the axis of
// revolution, as far from that end as it went past it. w = the cell index
// as stepped, n = the cell after clamping, changed here.
__device__ __forceinline__ bool pole_axis(int w, int nc, int ends, int& n) {
  if (w < 0 && (ends & 1)) {
    n = min(-w - 1, nc - 1);
    return true;
  }
  if (w >= nc && (ends & 2)) {
    n = max(2 * nc - 1 - w, 0);
    return true;
  }
  return false;
}

// Cell v in [0, nc) of a periodic axis, half a turn on.
__device__ __forceinline__ int half_turn(int v, int nc) {
  const int w = v + nc / 2;
  return w >= nc ? w - nc : w;
}

// Stencil walk in precision T from `cell`. On kFound, cell/s hold the donor.
// On kDoubt (T = float only), cell holds the cell where FP32 could not decide.
// perr bounds the error of each component of xi (FP32 only; 0 when exact).
// s_init: Newton's start in the first cell. Poles: a step clamped at a
// polar end that would revisit a cell goes on across the axis of
// revolution instead of ending the walk (else a point across the axis is
// left to the scan); on in the FP64 kernels, off in the mixed ones, whose
// registers it would push past two wavefronts per SIMD.
template <typename T, bool Poles = (sizeof(T) == 8)>
__device__ int walk(const GridDev& G, const uint8_t* fl, const double xi[3], double perr, int& cell, T s[3],
                    int max_walk, bool& limit, int& visited, int* iters = nullptr, const unsigned int* th = nullptr,
                    unsigned int stamp = 0, Start s_init = kCentre) {
  int ci, cj, ck;
  cell_ijk(G, cell, ci, cj, ck);
  int hist[4] = {-1, -1, -1, -1};  // the last cells visited: a revisit ends the walk
  // Newton starts in the first cell from s_init (or its centre); in each
  // later cell from the previous cell's s moved by the step taken (natural
  // coordinates of neighbouring cells continue across their shared face),
  // kept in [0, 1]
  s[0] = s_init.on ? (T)s_init.v[0] : (T)0.5;
  s[1] = s_init.on ? (T)s_init.v[1] : (T)0.5;
  s[2] = s_init.on ? (T)s_init.v[2] : (T)0.5;
  for (int stepn = 0; stepn < max_walk; ++stepn) {
    ++visited;
    CellMap<T> m;
    // FP64 (latency-bound sizes): the corner flags ride with the corner
    // coordinates; FP32 (the large batched sizes, bound by the gathers'
    // lines): only the accepted cell's flags are read
    uint8_t cf[8];
    bool hole_tile = true;
    if (sizeof(T) == 8) {
#pragma unroll
      for (int c = 0; c < 8; ++c) cf[c] = fl[corner_node(G, ci, cj, ck, c)];
    } else {
      // (issued with the corner loads; needed only if the cell is accepted)
      hole_tile = corner_tiles_hold_hole(G, ci, cj, ck, th, stamp);
    }
    load_cell<T>(G, ci, cj, ck, xi, m);
    T cond = 0, inv_norm = 0;
    bool conv =
        newton<T>(m, s, sizeof(T) == 4 ? &cond : (T*)nullptr, sizeof(T) == 4 ? &inv_norm : (T*)nullptr, iters);
    const int here = (int)((unsigned)ci + (unsigned)G.nci * ((unsigned)cj + (unsigned)G.ncj * (unsigned)ck));
    if (sizeof(T) == 4) {
      // FP32 decides only clear cases: inside with margin >= 1e-4 in a
      // well-conditioned cell, or outside by more than the FP32 error can
      // explain (then keep walking). Anything else goes to FP64 from here.
      T mg = fmin(fmin(s[0], (T)1 - s[0]), fmin(fmin(s[1], (T)1 - s[1]), fmin(s[2], (T)1 - s[2])));
      if (!(mg == mg)) {
        cell = here;
        return kDoubt;
      }
      const bool sure = conv && cond <= (T)kMixedCond;
      // the position error in natural coordinates, |ds|_inf <= ||J^-1||_2 |e|_2,
      // with e the query position's error (perr per component, twice over)
      // plus the corners' FP32 rounding (the map moves by at most pf_err
      // per component inside the cell, where the weights are a partition
      // of unity)
      const T es = (T)(1.7320508075688772 * (2.0 * perr + G.pf_err)) * inv_norm;
      if (sure && mg >= (T)kMixedMargin + es) {
        cell = here;
        return (!hole_tile || cell_valid(G, fl, ci, cj, ck)) ? kFound : kToScan;
      }
      if (mg > -((sure ? (T)kMixedMargin : (T)kClearlyOutside) + es)) {
        cell = here;
        return kDoubt;
      }
    } else {
      if (conv && inside<T>(s, (T)kSTol)) {
        cell = here;
        return (sizeof(T) == 8 ? corners_valid(cf) : (!hole_tile || cell_valid(G, fl, ci, cj, ck))) ? kFound : kToScan;
      }
    }
    if (!(s[0] == s[0] && s[1] == s[1] && s[2] == s[2])) return kToScan;
    // step toward the point by the integer part of s: up to a quarter turn
    // in a periodic direction (where s is an angle-like cell count, e.g. the
    // azimuth of a shell near its polar axis), up to 8 cells otherwise
    const int lim_i = (G.per & 1) ? max(2, G.nci / 4) : 8;
    const int lim_j = (G.per & 2) ? max(2, G.ncj / 4) : 8;
    const int lim_k = (G.per & 4) ? max(2, G.nck / 4) : 8;
    int di = 0, dj = 0, dk = 0;
    if (s[0] < (T)0) di = (int)fmax(-(T)lim_i, floor(s[0]));
    else if (s[0] > (T)1) di = (int)fmin((T)lim_i, floor(s[0]));
    if (s[1] < (T)0) dj = (int)fmax(-(T)lim_j, floor(s[1]));
    else if (s[1] > (T)1) dj = (int)fmin((T)lim_j, floor(s[1]));
    if (s[2] < (T)0) dk = (int)fmax(-(T)lim_k, floor(s[2]));
    else if (s[2] > (T)1) dk = (int)fmin((T)lim_k, floor(s[2]));
    bool clamped = false;
    int ni = step_axis(ci, di, G.nci, G.per & 1, clamped);
    int nj = step_axis(cj, dj, G.ncj, G.per & 2, clamped);
    int nk = step_axis(ck, dk, G.nck, G.per & 4, clamped);
    int next = (int)((unsigned)ni + (unsigned)G.nci * ((unsigned)nj + (unsigned)G.ncj * (unsigned)nk));
    hist[stepn & 3] = here;
    if (next == hist[0] || next == hist[1] || next == hist[2] || next == hist[3]) {
      // a step clamped at a polar end lands on a cell just visited: the
      // point lies across the axis of revolution, and the walk goes on
      // there, Newton from the cell's centre; any other revisit ends it
      if (!(Poles && G.pole)) return kToScan;
      bool across = pole_axis(ci + di, G.nci, G.pole & 3, ni);
      across |= pole_axis(cj + dj, G.ncj, (G.pole >> 2) & 3, nj);
      across |= pole_axis(ck + dk, G.nck, (G.pole >> 4) & 3, nk);
      if (!across) return kToScan;
      // (half a turn from the cell it stepped from: near the axis the
      // periodic natural coordinate says little about where the point lies)
      if (G.per & 1) ni = half_turn(ci, G.nci);
      else if (G.per & 2) nj = half_turn(cj, G.ncj);
      else nk = half_turn(ck, G.nck);
      next = (int)((unsigned)ni + (unsigned)G.nci * ((unsigned)nj + (unsigned)G.ncj * (unsigned)nk));
      if (next == hist[0] || next == hist[1] || next == hist[2] || next == hist[3]) return kToScan;
      s[0] = s[1] = s[2] = (T)0.5;
      di = dj = dk = 0;
    }
    s[0] = fmin(fmax(s[0] - (T)di, (T)0), (T)1);
    s[1] = fmin(fmax(s[1] - (T)dj, (T)0), (T)1);
    s[2] = fmin(fmax(s[2] - (T)dk, (T)0), (T)1);
    ci = ni;
    cj = nj;
    ck = nk;
  }
  limit = true;
  return kToScan;
}

// Sound rejection of a cell before Newton: the trilinear cell lies in the
// convex hull of its 8 corners, so a point whose projection on some axis
// falls outside the corners' projections (padded far beyond the containment
// tolerance) is in no part of the cell. Axes: x, y, z (the corner box) and
// the normals of the cell's mean i-, j- and k-faces, which separate
// neighbouring cells, including the thin polar wedges of shell grids.
__device__ __forceinline__ bool hull_excludes(const double P[8][3], const double xi[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double lo = P[0][d], hi = P[0][d];
#pragma unroll
    for (int c = 1; c < 8; ++c) {
      lo = fmin(lo, P[c][d]);
      hi = fmax(hi, P[c][d]);
    }
    double pad = 1e-9 * (hi - lo) + 1e-300;
    if (xi[d] < lo - pad || xi[d] > hi + pad) return true;
  }
  double ei[3], ej[3], ek[3], q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ei[d] = (P[1][d] - P[0][d]) + (P[3][d] - P[2][d]) + (P[5][d] - P[4][d]) + (P[7][d] - P[6][d]);
    ej[d] = (P[2][d] - P[0][d]) + (P[3][d] - P[1][d]) + (P[6][d] - P[4][d]) + (P[7][d] - P[5][d]);
    ek[d] = (P[4][d] - P[0][d]) + (P[5][d] - P[1][d]) + (P[6][d] - P[2][d]) + (P[7][d] - P[3][d]);
    q[d] = xi[d] - P[0][d];
  }
  double n[3][3] = {{ej[1] * ek[2] - ej[2] * ek[1], ej[2] * ek[0] - ej[0] * ek[2], ej[0] * ek[1] - ej[1] * ek[0]},
                    {ek[1] * ei[2] - ek[2] * ei[1], ek[2] * ei[0] - ek[0] * ei[2], ek[0] * ei[1] - ek[1] * ei[0]},
                    {ei[1] * ej[2] - ei[2] * ej[1], ei[2] * ej[0] - ei[0] * ej[2], ei[0] * ej[1] - ei[1] * ej[0]}};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double lo = 0.0, hi = 0.0;  // corner 0 projects to 0
#pragma unroll
    for (int c = 1; c < 8; ++c) {
      double v = n[a][0] * (P[c][0] - P[0][0]) + n[a][1] * (P[c][1] - P[0][1]) + n[a][2] * (P[c][2] - P[0][2]);
      lo = fmin(lo, v);
      hi = fmax(hi, v);
    }
    double pq = n[a][0] * q[0] + n[a][1] * q[1] + n[a][2] * q[2];
    double pad = 1e-9 * (hi - lo) + 1e-300;
    if (pq < lo - pad || pq > hi + pad) return true;
  }
  return false;
}

// Candidate donor grid at position t of a query of grid A: t = -2 the cause
// grid, t = -1 the background, t >= 0 grid t; -1 where that position is
// skipped (Sec. 2.4 item 1).
__device__ __forceinline__ int candidate_at(int t, int A, int first) {
  if (t == -2) return first;
  if (t == -1) return (A == 0 || first == 0) ? -1 : 0;
  if (t == A || t == first || (t == 0 && A != 0)) return -1;
  return t;
}

struct Query {
  int A, cause, first;
  long long key, m;
  double x[3];
  double err;  // bound on the error of each component of x (0: x is exact)
  bool finite;
};

// Inertial position of a node from its FP64 body-frame coordinates.
__device__ __forceinline__ void world_of(const double* pa, double X, double Y, double Z, double x[3]) {
  x[0] = pa[0] * X + pa[1] * Y + pa[2] * Z + pa[9];
  x[1] = pa[3] * X + pa[4] * Y + pa[5] * Z + pa[10];
  x[2] = pa[6] * X + pa[7] * Y + pa[8] * Z + pa[11];
}

// Inertial position of node m of grid A, in FP64 from its FP64 coordinates.
__device__ __forceinline__ void exact_world(const GridDev& GA, const double* pa, long long m, double x[3]) {
  double X, Y, Z;
  load_xyz(GA, m, X, Y, Z);
  world_of(pa, X, Y, Z, x);
}

// The query of grid A's node m with its offset (o0, o1, o2) from the
// transform (x - c_A), from the node's flag byte and, where the position is
// taken in FP64 (exact, or the background in FP32), its coordinates
// (X, Y, Z).
template <typename T>
__device__ __forceinline__ Query query_from(const GridDev* __restrict__ grids, int ngrids, const double* sp, int A,
                                            long long m, uint8_t flag, double o0, double o1, double o2, bool exact,
                                            double X, double Y, double Z) {
  Query Q;
  Q.A = A;
  Q.m = m;
  Q.key = grids[Q.A].node_off + Q.m;
  Q.cause = flag >> 2;
  Q.first = (Q.cause != OV_CAUSE_BOUNDARY && Q.cause != Q.A && Q.cause < ngrids) ? Q.cause : -1;
  const double* pa = sp + 12 * Q.A;
  Q.err = 0.0;
  if (sizeof(T) == 4 && (exact || Q.A == 0)) {
    // the background's offsets are absolute positions (large, so FP32 would
    // lose most of a cell); take them in FP64
    world_of(pa, X, Y, Z, Q.x);
  } else {
    Q.x[0] = pa[9] + o0;
    Q.x[1] = pa[10] + o1;
    Q.x[2] = pa[11] + o2;
    // FP32 transform from FP32 coordinates and pose: a few roundings of
    // terms no larger than |X|_1 <= sqrt(3) |qx|_2 <= sqrt(3) |qx|_1 each
    if (sizeof(T) == 4) Q.err = ldexp(fabs(o0) + fabs(o1) + fabs(o2), -20);
  }
  Q.finite = isfinite(Q.x[0]) && isfinite(Q.x[1]) && isfinite(Q.x[2]);
  return Q;
}

// The query of grid A's node m (query_from), its flag and coordinates read
// here. exact = true (or the background in FP32) takes the position from the
// FP64 node coordinates instead of the transform's FP32 output.
template <typename T>
__device__ __forceinline__ Query make_query(const GridDev* __restrict__ grids, int ngrids, const double* sp,
                                            const uint8_t* __restrict__ flags, int A, long long m, double o0,
                                            double o1, double o2, bool exact) {
  const GridDev& GA = grids[A];
  const uint8_t flag = flags[GA.node_off + m];
  double X = 0.0, Y = 0.0, Z = 0.0;
  if (sizeof(T) == 4 && (exact || A == 0)) load_xyz(GA, m, X, Y, Z);
  return query_from<T>(grids, ngrids, sp, A, m, flag, o0, o1, o2, exact, X, Y, Z);
}

// Query q of the list, its offset read from the transform's output qx.
template <typename T>
__device__ __forceinline__ Query load_query(const GridDev* __restrict__ grids, int ngrids, const double* sp,
                                            const uint8_t* __restrict__ flags, const int32_t* __restrict__ q_grid,
                                            const int32_t* __restrict__ q_node, const T* __restrict__ qx,
                                            long long cap, long long q, bool exact = false) {
  const int A = q_grid[q];
  const bool need = !(sizeof(T) == 4 && (exact || A == 0));
  const double o0 = need ? (double)qx[q] : 0.0, o1 = need ? (double)qx[cap + q] : 0.0,
               o2 = need ? (double)qx[2 * cap + q] : 0.0;
  return make_query<T>(grids, ngrids, sp, flags, A, q_node[q], o0, o1, o2, exact);
}

__device__ __forceinline__ void body_frame(const double* pb, const double x[3], double xi[3]) {
  double d0 = x[0] - pb[9], d1 = x[1] - pb[10], d2 = x[2] - pb[11];
  xi[0] = pb[0] * d0 + pb[3] * d1 + pb[6] * d2;
  xi[1] = pb[1] * d0 + pb[4] * d1 + pb[7] * d2;
  xi[2] = pb[2] * d0 + pb[5] * d1 + pb[8] * d2;
}

// Query position in grid B's body frame; false if outside the box of B's
// nodes (padded by the position's error bound).
__device__ __forceinline__ bool to_body(const GridDev& G, const double* pb, const Query& Q, double xi[3]) {
  body_frame(pb, Q.x, xi);
  double ext = fmax(G.bhi[0] - G.blo[0], fmax(G.bhi[1] - G.blo[1], G.bhi[2] - G.blo[2]));
  double pad = 1e-8 * ext + 2.0 * Q.err;
  return !(xi[0] < G.blo[0] - pad || xi[0] > G.bhi[0] + pad || xi[1] < G.blo[1] - pad || xi[1] > G.bhi[1] + pad ||
           xi[2] < G.blo[2] - pad || xi[2] > G.bhi[2] + pad);
}

// The exact FP64 position in B's frame (xi itself when it is already exact).
__device__ __forceinline__ void exact_body(const GridDev* grids, const double* sp, const Query& Q, int B,
                                           const double xi[3], double xe[3]) {
  if (Q.err == 0.0) {
    xe[0] = xi[0];
    xe[1] = xi[1];
    xe[2] = xi[2];
    return;
  }
  double x[3];
  exact_world(grids[Q.A], sp + 12 * Q.A, Q.m, x);
  body_frame(sp + 12 * B, x, xe);
}

__device__ __forceinline__ long long bin_of(const GridDev& G, const double xi[3]) {
  return bin_axis(G, 0, xi[0]) +
         (long long)G.nb[0] * (bin_axis(G, 1, xi[1]) + (long long)G.nb[1] * bin_axis(G, 2, xi[2]));
}

// Walk in grid B from `seed` (FP32 first in mixed precision, then FP64 on the
// exact position from any cell FP32 cannot decide). Returns kFound with
// cell/s, else kToScan.
template <typename T>
__device__ __forceinline__ int walk_grid(const GridDev* grids, const double* sp, const Query& Q, int B,
                                         const uint8_t* fl, const double xi[3], int& cell, T s[3], int max_walk,
                                         bool& limit, int& how, int& visited, int* iters = nullptr) {
  const GridDev& G = grids[B];
  int r = walk<T>(G, fl, xi, Q.err, cell, s, max_walk, limit, visited, iters);
  if (sizeof(T) == 4 && r == kDoubt) {
    double s64[3], xe[3];
    exact_body(grids, sp, Q, B, xi, xe);
    r = walk<double, sizeof(T) == 8>(G, fl, xe, 0.0, cell, s64, max_walk, limit, visited, iters, nullptr, 0u,
                                     start_from<T>(s));
    s[0] = (T)s64[0];
    s[1] = (T)s64[1];
    s[2] = (T)s64[2];
    how |= OV_Q_FP64_FIXED;
  }
  return r;
}

// Warm-start history: per node, the donor (grid, cell) of its last query,
// its natural coordinates to 5 bits each (the next step's Newton start in
// that cell) and the low byte of the stamp of the step that wrote it, in
// one 8-byte record. A node that was not a query in the last steps (one that just
// entered the buffer layer, say) would start its walk from a donor long out
// of date; its entry is then ignored and the walk starts from the control
// cell's seed.
struct Warm {
  unsigned long long* rec;
  const unsigned int* stamp;  // the running step's stamp
  int use;
};
constexpr int kWarmMaxAge = 2;  // steps

// The node's warm seed from its record r: grid (255: none), cell and the
// Newton start there.
__device__ __forceinline__ void warm_decode(const Warm& w, unsigned long long r, uint8_t now, int& grid, int& cell,
                                            Start& s0) {
  grid = 255;
  cell = -1;
  s0 = kCentre;
  if (!w.use) return;
  const uint8_t age = (uint8_t)(now - (uint8_t)(r >> 40));
  if (age > kWarmMaxAge) return;
  grid = (int)((r >> 32) & 0xFF);
  cell = (int)(uint32_t)r;
  const unsigned int b = (unsigned int)(r >> 48);
  s0.on = true;
  s0.v[0] = (double)(b & 31u) * (1.0 / 31.0);
  s0.v[1] = (double)((b >> 5) & 31u) * (1.0 / 31.0);
  s0.v[2] = (double)((b >> 10) & 31u) * (1.0 / 31.0);
}

__device__ __forceinline__ void warm_read(const Warm& w, long long key, uint8_t now, int& grid, int& cell,
                                          Start& s0) {
  warm_decode(w, w.use ? gp(w.rec)[key] : 0ull, now, grid, cell, s0);
}

// What the first round trip of a query brings: its node's FP64 coordinates
// (the gather layout), its warm-start record and its flag byte. The back
// kernel loads them a chunk ahead.
struct NodePre {
  double x, y, z;
  unsigned long long rec;
  uint32_t flag;
};

__device__ __forceinline__ void node_pre_load(const GridDev& G, const Warm& w, const uint8_t* __restrict__ flags,
                                              int m, NodePre& p) {
  load_xyz(G, m, p.x, p.y, p.z);
  const long long key = G.node_off + m;
  p.rec = w.use ? gp(w.rec)[key] : 0ull;
  p.flag = flags[key];
}

// s to 5 bits per component (nearest of 0, 1/31, ..., 1; a NaN as 1/2).
template <typename T>
__device__ __forceinline__ unsigned long long warm_s_bits(const T s[3]) {
  const Start v = start_from<T>(s);
  unsigned long long b = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) b |= (unsigned long long)(unsigned int)rint(v.v[d] * 31.0) << (5 * d);
  return b << 48;
}

template <typename T>
__device__ __forceinline__ void write_result(long long q, long long cap, long long key, int grid, int cell, int st,
                                             const T s[3], int32_t* donor_grid, int32_t* donor_cell, T* s_out,
                                             int32_t* status, const Warm& warm, uint8_t now) {
  donor_grid[q] = grid;
  donor_cell[q] = cell;
  status[q] = st;  // bits 8-15: cells the walk visited (diagnostic)
  s_out[q] = s[0];
  s_out[cap + q] = s[1];
  s_out[2 * cap + q] = s[2];
  warm.rec[key] = (unsigned long long)(uint32_t)cell | ((unsigned long long)(grid < 0 ? 255u : (unsigned)grid) << 32) |
                  ((unsigned long long)now << 40) | warm_s_bits<T>(s);
}

// Markers left in donor_grid between the passes of one search call; status
// then holds the candidate position t + 2 (bits 0-7) and the cells visited
// so far (bits 8-15), donor_cell the cell to continue from.
constexpr int kDeferFix = -2;   // FP32 could not decide: the FP64 correction continues
constexpr int kDeferScan = -3;  // the walk failed: brute-force scan from candidate t

__device__ __forceinline__ int defer_status(int t, int visited) { return (t + 2) | (min(visited, 255) << 8); }

// Pass 1: one query per lane, the walk in T over the candidate grids. The
// first grid whose walk finds a valid containing cell is the donor; a walk
// FP32 cannot decide or that fails is deferred to the passes below, which
// keep its place in the candidate order.
template <typename T>
__global__ void __launch_bounds__(256)
    k_donor_walk(const GridDev* __restrict__ grids, int ngrids, const double* __restrict__ poses,
                 const uint8_t* __restrict__ flags, const int32_t* __restrict__ q_grid,
                 const int32_t* __restrict__ q_node, const T* __restrict__ qx, const long long* __restrict__ d_count,
                 long long cap, int32_t* __restrict__ donor_grid, int32_t* __restrict__ donor_cell,
                 T* __restrict__ s_out, int32_t* __restrict__ status, Warm warm, int max_walk,
                 int32_t* __restrict__ dev_status) {
  __shared__ double sp[kMaxGrids * 12];
  for (int i = threadIdx.x; i < ngrids * 12; i += blockDim.x) sp[i] = poses[i];
  const uint8_t now = (uint8_t)*warm.stamp;
  __syncthreads();
  const long long n = min(*d_count, cap);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    const Query Q = load_query<T>(grids, ngrids, sp, flags, q_grid, q_node, qx, cap, q);
    int res_grid = -1, res_cell = -1, res_status = OV_Q_ORPHAN;
    T rs[3] = {(T)NAN, (T)NAN, (T)NAN};
    bool limit = false;
    int visited = 0, defer = 0, defer_t = 0;
    T s[3] = {(T)NAN, (T)NAN, (T)NAN};
    if (!Q.finite) {
      atomicOr(dev_status, OV_DEV_NONFINITE);
    } else {
      int wg, wc;
      Start ws;
      warm_read(warm, Q.key, now, wg, wc, ws);
      for (int t = -2; t < ngrids; ++t) {
        const int B = candidate_at(t, Q.A, Q.first);
        if (B < 0) continue;
        const GridDev& G = grids[B];
        double xi[3];
        if (!to_body(G, sp + 12 * B, Q, xi)) continue;
        // seeds: last step's donor cell, then the control cell's lowest cell
        const int rep = gp(G.brep)[bin_of(G, xi)];
        int seed = -1;
        if (wg == B && wc >= 0 && (long long)wc < G.ncells) seed = wc;
        if (seed < 0 && rep < 0) continue;  // no cell reaches this control cell
        int cell = seed >= 0 ? seed : rep;
        int r = walk<T>(G, flags + G.node_off, xi, Q.err, cell, s, max_walk, limit, visited, nullptr, nullptr, 0u,
                        seed >= 0 ? ws : kCentre);
        if (r == kToScan && seed >= 0 && rep >= 0 && rep != seed) {
          cell = rep;  // a second start before the brute-force scan
          r = walk<T>(G, flags + G.node_off, xi, Q.err, cell, s, max_walk, limit, visited);
        }
        if (r == kFound) {
          res_grid = B;
          res_cell = cell;
          res_status = OV_Q_FOUND;
          rs[0] = s[0];
          rs[1] = s[1];
          rs[2] = s[2];
        } else {
          defer = r == kDoubt ? kDeferFix : kDeferScan;
          defer_t = t;
          res_cell = cell;
        }
        break;
      }
    }
    if (limit) atomicOr(dev_status, OV_DEV_WALK_LIMIT);
    if (defer) {
      donor_grid[q] = defer;
      donor_cell[q] = res_cell;
      status[q] = defer_status(defer_t, visited);
      if (defer == kDeferFix) {  // the FP32 solve's s: the FP64 correction's start
        s_out[q] = s[0];
        s_out[cap + q] = s[1];
        s_out[2 * cap + q] = s[2];
      }
    } else {
      write_result<T>(q, cap, Q.key, res_grid, res_cell, res_status | (min(visited, 255) << 8), rs, donor_grid,
                      donor_cell, s_out, status, warm, now);
    }
  }
}

// Pass 2 (mixed precision): the FP64 correction. One query per lane; for each
// query FP32 could not decide, the walk continues in FP64 from that cell on
// the query's exact position (recomputed from the FP64 node coordinates).
__global__ void __launch_bounds__(256)
    k_donor_fix(const GridDev* __restrict__ grids, int ngrids, const double* __restrict__ poses,
                const uint8_t* __restrict__ flags, const int32_t* __restrict__ q_grid,
                const int32_t* __restrict__ q_node, const float* __restrict__ qx, const long long* __restrict__ d_count,
                long long cap, int32_t* __restrict__ donor_grid, int32_t* __restrict__ donor_cell,
                float* __restrict__ s_out, int32_t* __restrict__ status, Warm warm, int max_walk,
                int32_t* __restrict__ dev_status) {
  __shared__ double sp[kMaxGrids * 12];
  for (int i = threadIdx.x; i < ngrids * 12; i += blockDim.x) sp[i] = poses[i];
  const uint8_t now = (uint8_t)*warm.stamp;
  __syncthreads();
  const long long n = min(*d_count, cap);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    if (donor_grid[q] != kDeferFix) continue;
    const int st = status[q];
    const int t = (st & 255) - 2;
    int visited = (st >> 8) & 255;
    const Query Q = load_query<float>(grids, ngrids, sp, flags, q_grid, q_node, qx, cap, q, true);
    const int B = candidate_at(t, Q.A, Q.first);
    const GridDev& G = grids[B];
    double xi[3], s64[3];
    body_frame(sp + 12 * B, Q.x, xi);
    int cell = donor_cell[q];
    bool limit = false;
    const float sf0[3] = {s_out[q], s_out[cap + q], s_out[2 * cap + q]};
    const int r = walk<double, false>(G, flags + G.node_off, xi, 0.0, cell, s64, max_walk, limit, visited, nullptr,
                                      nullptr, 0u, start_from<float>(sf0));
    if (limit) atomicOr(dev_status, OV_DEV_WALK_LIMIT);
    if (r == kFound) {
      const float sf[3] = {(float)s64[0], (float)s64[1], (float)s64[2]};
      write_result<float>(q, cap, Q.key, B, cell, OV_Q_FOUND | OV_Q_FP64_FIXED | (min(visited, 255) << 8), sf,
                          donor_grid, donor_cell, s_out, status, warm, now);
    } else {
      donor_grid[q] = kDeferScan;
      status[q] = defer_status(t, visited);
    }
  }
}

// Block-cooperative brute-force scan of the control cell (or sub-bin)
// holding xi: its sorted list is taken blockDim.x candidates per round, one
// per thread; the first round holding a valid containing cell ends the scan
// with its lowest such cell (lists ascend, so that is the lowest list
// position that hits). Every cell containing xi is on that list, so this is
// the lowest valid containing cell of the grid.
// The next round's cell ids are loaded while the current round is tested.
// Every thread of the block calls it with the same G and xi.
struct ScanLds {
  int pos[4];
  int cell[4];
  double s[4][3];
};

// *cands / *iters (if given) are increased by this thread's tested list
// entries and Newton iterations.
__device__ int scan_control_cell_block(const GridDev& G, const uint8_t* fl, const double xi[3], double s_best[3],
                                       ScanLds& S, int* cands = nullptr, int* iters = nullptr) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  long long e0, e1;
  gmem<int>* list = gp(control_list(G, xi, e0, e1));
  int next = e0 + tid < e1 ? list[e0 + tid] : -1;
  for (long long base = e0; base < e1; base += blockDim.x) {
    const long long e = base + tid;
    const int cell = next;
    next = e + blockDim.x < e1 ? list[e + blockDim.x] : -1;
    bool hit = false;
    double s[3] = {0.0, 0.0, 0.0};
    if (e < e1) {
      if (cands) ++*cands;
      int ci, cj, ck;
      cell_ijk(G, cell, ci, cj, ck);
      double P[8][3];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        load_xyz(G, corner_node(G, ci, cj, ck, c), P[c][0], P[c][1], P[c][2]);
      }
      if (!hull_excludes(P, xi)) {
        CellMap<double> m;
        map_from_corners<double>(P, xi, m);
        s[0] = s[1] = s[2] = 0.5;
        hit = newton<double>(m, s, nullptr, nullptr, iters) && inside<double>(s, kSTol) && cell_valid(G, fl, ci, cj, ck);
      }
    }
    const unsigned long long hits = __ballot(hit);
    const int first = hits ? __ffsll((long long)hits) - 1 : 64;
    if (lane == first) {
      S.pos[wave] = tid;
      S.cell[wave] = cell;
      S.s[wave][0] = s[0];
      S.s[wave][1] = s[1];
      S.s[wave][2] = s[2];
    }
    if (lane == 0 && !hits) S.pos[wave] = 0x7fffffff;
    __syncthreads();
    int bw = -1, bp = 0x7fffffff;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
      if (S.pos[w] < bp) {
        bp = S.pos[w];
        bw = w;
      }
    int found = -1;
    if (bw >= 0) {
      found = S.cell[bw];
      s_best[0] = S.s[bw][0];
      s_best[1] = S.s[bw][1];
      s_best[2] = S.s[bw][2];
    }
    __syncthreads();  // S is reused by the next round or call
    if (found >= 0) return found;
  }
  return -1;
}

// The same scan by one wavefront: 64 candidates per round; the first hit in
// list order (the lowest cell index) is taken from its lane by shuffles, so
// the wavefront needs no barrier and no shared memory.
__device__ int scan_control_cell_wave(const GridDev& G, const uint8_t* fl, const double xi[3], double s_best[3],
                                      int* cands = nullptr, int* iters = nullptr) {
  const int lane = threadIdx.x & 63;
  long long e0, e1;
  gmem<int>* list = gp(control_list(G, xi, e0, e1));
  int next = e0 + lane < e1 ? list[e0 + lane] : -1;
  for (long long base = e0; base < e1; base += 64) {
    const long long e = base + lane;
    const int cell = next;
    next = e + 64 < e1 ? list[e + 64] : -1;
    bool hit = false;
    double s[3] = {0.0, 0.0, 0.0};
    if (e < e1) {
      if (cands) ++*cands;
      int ci, cj, ck;
      cell_ijk(G, cell, ci, cj, ck);
      double P[8][3];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        load_xyz(G, corner_node(G, ci, cj, ck, c), P[c][0], P[c][1], P[c][2]);
      }
      if (!hull_excludes(P, xi)) {
        CellMap<double> m;
        map_from_corners<double>(P, xi, m);
        s[0] = s[1] = s[2] = 0.5;
        hit = newton<double>(m, s, nullptr, nullptr, iters) && inside<double>(s, kSTol) && cell_valid(G, fl, ci, cj, ck);
      }
    }
    const unsigned long long hits = __ballot(hit);
    if (hits) {  // (the same in every lane)
      const int first = __ffsll((long long)hits) - 1;
      s_best[0] = __shfl(s[0], first, 64);
      s_best[1] = __shfl(s[1], first, 64);
      s_best[2] = __shfl(s[2], first, 64);
      return __shfl(cell, first, 64);
    }
  }
  return -1;
}

// Pass 3: the brute-force scan (Alg. 3's fallback). Each block sweeps 256
// queries, lists the deferred ones (with their status) in LDS, and takes
// them one at a time with all its threads: the cooperative scan of the grid
// whose walk failed, then the remaining candidate grids (walk, and
// cooperative scan if needed), all on the exact query position.
template <typename T>
__global__ void __launch_bounds__(256)
    k_donor_scan(const GridDev* __restrict__ grids, int ngrids, const double* __restrict__ poses,
                 const uint8_t* __restrict__ flags, const int32_t* __restrict__ q_grid,
                 const int32_t* __restrict__ q_node, const T* __restrict__ qx, const long long* __restrict__ d_count,
                 long long cap, int32_t* __restrict__ donor_grid, int32_t* __restrict__ donor_cell,
                 T* __restrict__ s_out, int32_t* __restrict__ status, Warm warm, int max_walk,
                 int32_t* __restrict__ dev_status) {
  __shared__ double sp[kMaxGrids * 12];
  __shared__ int list_q[256], list_st[256];
  __shared__ int nlist;
  __shared__ ScanLds S;
  for (int i = threadIdx.x; i < ngrids * 12; i += blockDim.x) sp[i] = poses[i];
  const uint8_t now = (uint8_t)*warm.stamp;
  const long long n = min(*d_count, cap);
  for (long long base = (long long)blockIdx.x * blockDim.x; base < n; base += (long long)gridDim.x * blockDim.x) {
    if (threadIdx.x == 0) nlist = 0;
    __syncthreads();
    const long long ql = base + threadIdx.x;
    if (ql < n && donor_grid[ql] == kDeferScan) {
      const int slot = atomicAdd(&nlist, 1);
      list_q[slot] = (int)threadIdx.x;
      list_st[slot] = status[ql];
    }
    __syncthreads();
    const int nd = nlist;
    for (int d = 0; d < nd; ++d) {
      const long long q = base + list_q[d];
      const int st = list_st[d];
      const int t0 = (st & 255) - 2;
      int visited = (st >> 8) & 255;
      const Query Q = load_query<T>(grids, ngrids, sp, flags, q_grid, q_node, qx, cap, q, true);
      int res_grid = -1, res_cell = -1, res_status = OV_Q_ORPHAN;
      T rs[3] = {(T)NAN, (T)NAN, (T)NAN};
      bool limit = false;
      for (int t = t0; t < ngrids; ++t) {
        const int B = candidate_at(t, Q.A, Q.first);
        if (B < 0) continue;
        const GridDev& G = grids[B];
        double xi[3];
        if (t == t0) body_frame(sp + 12 * B, Q.x, xi);  // the deferred grid passed the box test
        else if (!to_body(G, sp + 12 * B, Q, xi)) continue;
        const uint8_t* fl = flags + G.node_off;
        int cell = -1, how = OV_Q_FALLBACK;
        T s[3];
        bool walked = false;
        if (t != t0) {
          int seed = gp(G.brep)[bin_of(G, xi)];
          if (seed < 0) continue;
          cell = seed;
          how = OV_Q_FOUND;
          walked = walk_grid<T>(grids, sp, Q, B, fl, xi, cell, s, max_walk, limit, how, visited) == kFound;
        }
        if (!walked) {
          double s64[3];
          cell = scan_control_cell_block(G, fl, xi, s64, S);
          s[0] = (T)s64[0];
          s[1] = (T)s64[1];
          s[2] = (T)s64[2];
          how = OV_Q_FALLBACK;
        }
        if (cell >= 0) {
          res_grid = B;
          res_cell = cell;
          res_status = how;
          rs[0] = s[0];
          rs[1] = s[1];
          rs[2] = s[2];
          break;
        }
      }
      if (threadIdx.x == 0) {
        if (limit) atomicOr(dev_status, OV_DEV_WALK_LIMIT);
        write_result<T>(q, cap, Q.key, res_grid, res_cell, res_status | (min(visited, 255) << 8), rs, donor_grid,
                        donor_cell, s_out, status, warm, now);
      }
    }
    __syncthreads();  // the list is rebuilt for the next range
  }
}

// Queue of the two-kernel back half: the queries the first kernel could not
// decide (an FP32 walk left in doubt, or a walk that must hand over to the
// brute-force scan), as indices into the step's query list. Their state is
// kept in the step's outputs meanwhile, as between the passes of the search
// call: donor_grid a marker, donor_cell the cell to go on from, status the
// candidate position and the cells visited. Two counters serve alternate
// steps (the parity of the step's stamp): a step's first kernel appends to
// its own and clears the other, which the previous step's second kernel has
// finished reading (the back halves of consecutive steps run in stream
// order).
// `chunk` (optional, [2], the same parity rule): the work queue's heads.
// With it, a block takes its first BS-query chunk by its index and each
// further one from an atomic head (the grid's chunks after its own
// first), asked for at the start of the chunk before, so that blocks that
// meet cheap queries take more chunks.
struct DeferQueue {
  int32_t* items;        // [capacity]
  unsigned int* count;   // [2]
  unsigned int* chunk;   // [2] or null: static chunks (block b takes b, b + grid, ...)
};

// The cooperative scans of a block's deferred queries, one query at a time
// with all the block's threads (Alg. 3's fallback): the scan of the grid whose
// walk failed, then the remaining candidate grids (walk, and scan where it
// fails), all on the exact query position. Entry d of the LDS list is query
// list_q[d] of thread list_owner[d] with deferral status list_st[d]; the
// owner thread receives the result. The same rules as the scan pass of the
// search call.
// One deferred query (position t0 of its candidate list, `dvisited` cells
// walked so far), taken by every thread of the group that scans: the exact
// position in FP64; in the grid of position t0 the brute-force scan of the
// control cell; in later grids a walk from the control cell's seed, and the
// scan if the walk fails. The first grid with a valid containing cell is
// the donor. WAVE: the scans run on one wavefront (else the whole block).
template <typename T, bool WAVE>
__device__ __forceinline__ void deferred_scan_one(const GridDev* __restrict__ grids, int ngrids, const double* sp,
                                                  const uint8_t* __restrict__ flags, int A, int qm, int st,
                                                  ScanLds& S, int max_walk, int& g_grid, int& g_cell,
                                                  int& g_status, T gs[3], int& dvisited, bool& dlimit,
                                                  int& walk_iters, int& my_iters, int& my_cands) {
  const int t0 = (st & 255) - 2;
  dvisited = (st >> 8) & 255;
  T o[3] = {0, 0, 0};
  if (sizeof(T) == 8) transform_node<T>(grids[A], sp + 12 * A, qm, o);  // (FP32: the exact position)
  const Query Q = make_query<T>(grids, ngrids, sp, flags, A, qm, (double)o[0], (double)o[1], (double)o[2], true);
  g_grid = -1;
  g_cell = -1;
  g_status = OV_Q_ORPHAN;
  gs[0] = gs[1] = gs[2] = (T)NAN;
  for (int t = t0; t < ngrids; ++t) {
    const int B = candidate_at(t, Q.A, Q.first);
    if (B < 0) continue;
    const GridDev& G = grids[B];
    double xi[3];
    if (t == t0) body_frame(sp + 12 * B, Q.x, xi);
    else if (!to_body(G, sp + 12 * B, Q, xi)) continue;
    const uint8_t* fl = flags + G.node_off;
    int cell = -1, how = OV_Q_FALLBACK;
    T s[3];
    bool walked = false;
    if (t != t0) {
      int seed = gp(G.brep)[bin_of(G, xi)];
      if (seed < 0) continue;
      cell = seed;
      how = OV_Q_FOUND;
      walked = walk_grid<T>(grids, sp, Q, B, fl, xi, cell, s, max_walk, dlimit, how, dvisited, &walk_iters) == kFound;
    }
    if (!walked) {
      double s64[3];
      cell = WAVE ? scan_control_cell_wave(G, fl, xi, s64, &my_cands, &my_iters)
                  : scan_control_cell_block(G, fl, xi, s64, S, &my_cands, &my_iters);
      s[0] = (T)s64[0];
      s[1] = (T)s64[1];
      s[2] = (T)s64[2];
      how = OV_Q_FALLBACK;
    }
    if (cell >= 0) {
      g_grid = B;
      g_cell = cell;
      g_status = how;
      gs[0] = s[0];
      gs[1] = s[1];
      gs[2] = s[2];
      break;
    }
  }
}

template <typename T>
__device__ __forceinline__ void block_deferred_scans(const GridDev* __restrict__ grids, int ngrids, const double* sp,
                                                     const uint8_t* __restrict__ flags,
                                                     const int32_t* __restrict__ q_grid,
                                                     const int32_t* __restrict__ q_node, int nd,
                                                     const int* list_owner, const long long* list_q,
                                                     const int* list_st, ScanLds& S, int max_walk, int& res_grid,
                                                     int& res_cell, int& res_status, T rs[3], int& visited,
                                                     bool& limit, int& my_iters, int& my_cands) {
  for (int d = 0; d < nd; ++d) {
    // every thread takes the deferred query (same values in all lanes)
    const int owner = list_owner[d];
    const long long qd = list_q[d];
    int g_grid, g_cell, g_status, dvisited, walk_iters = 0;  // (walk work counted once, by the owner)
    T gs[3];
    bool dlimit = false;
    deferred_scan_one<T, false>(grids, ngrids, sp, flags, q_grid[qd], q_node[qd], list_st[d], S, max_walk, g_grid,
                                g_cell, g_status, gs, dvisited, dlimit, walk_iters, my_iters, my_cands);
    if ((int)threadIdx.x == owner) {
      res_grid = g_grid;
      res_cell = g_cell;
      res_status = g_status;
      rs[0] = gs[0];
      rs[1] = gs[1];
      rs[2] = gs[2];
      visited = dvisited;
      limit |= dlimit;
      my_iters += walk_iters;
    }
  }
}

// A query's result written out (donor, natural coordinates, status, warm-start
// record) and its four fields interpolated (turned into the receiver's frame
// when asked).
template <typename T>
__device__ __forceinline__ void finish_query(const GridDev* __restrict__ grids, const double* sp, long long q,
                                             long long cap, long long key, int my_grid, int res_grid, int res_cell,
                                             int res_status, int visited, const T rs[3],
                                             int32_t* __restrict__ donor_grid, int32_t* __restrict__ donor_cell,
                                             T* __restrict__ s_out, int32_t* __restrict__ status, const Warm& warm,
                                             uint8_t now, const T* __restrict__ fields, long long total_nodes,
                                             int interleaved, int frame_velocity, T* __restrict__ out) {
  write_result<T>(q, cap, key, res_grid, res_cell, res_status | (min(visited, 255) << 8), rs, donor_grid, donor_cell,
                  s_out, status, warm, now);
  if (fields && res_grid >= 0) {
    T v[4];
    interp_point<T>(grids[res_grid], res_cell, rs[0], rs[1], rs[2], fields, total_nodes, interleaved != 0, v);
    if (frame_velocity) frame_rotate<T>(sp + 12 * my_grid, sp + 12 * res_grid, v);
#pragma unroll
    for (int f = 0; f < 4; ++f) out[(long long)f * cap + q] = v[f];
  }
}

// The wavefront's work counters, summed across its lanes with shuffles (an
// atomic on a value that differs per lane compiles to a serial loop over the
// lanes), then one device atomic per counter from its first lane.
__device__ __forceinline__ void add_work_counters(unsigned long long* stats, unsigned int cells, unsigned int iters,
                                                  unsigned int cands) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    cells += __shfl_xor(cells, o, 64);
    iters += __shfl_xor(iters, o, 64);
    cands += __shfl_xor(cands, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    unsigned long long* slot = stat_slot(stats);
    if (cells) atomicAdd(&slot[OV_STAT_SEARCH_CELLS], (unsigned long long)cells);
    if (iters) atomicAdd(&slot[OV_STAT_NEWTON_ITERS], (unsigned long long)iters);
    if (cands) atomicAdd(&slot[OV_STAT_SCAN_CANDIDATES], (unsigned long long)cands);
  }
}

// Occupancy asked of the walk kernel of the two-kernel back half: with the
// cold paths in the second kernel, the FP32 walk fits three wavefronts per
// SIMD (168 VGPRs).
template <typename T>
struct WalkWaves {
  static constexpr int value = sizeof(T) == 4 ? 3 : 1;
};

// The first kernel of the two-kernel back half (OV_OPT_BACK_FUSED = 2). Each
// wavefront takes 64 queries at a time, one per lane (by a fixed stride over
// all the launch's wavefronts, or from the work queue), with no barrier
// between wavefronts: the transform and the walk over the candidate grids.
// A query FP32 cannot decide, or whose walk fails, goes to the deferral queue
// (its state in its outputs) for k_back_defer; every other lane writes its
// result and interpolates its fields. The kernel holds only the walk's
// registers, which leaves room for three wavefronts per SIMD in FP32.
template <typename T, int BS>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(WalkWaves<T>::value)))
    k_back_walk(const GridDev* __restrict__ grids_g, int ngrids, const double* __restrict__ poses,
           const uint8_t* __restrict__ flags, const int32_t* __restrict__ q_grid, const int32_t* __restrict__ q_node,
           T* __restrict__ qx, const long long* __restrict__ d_count, long long cap,
           int32_t* __restrict__ donor_grid, int32_t* __restrict__ donor_cell, T* __restrict__ s_out,
           int32_t* __restrict__ status, Warm warm, int max_walk, int32_t* __restrict__ dev_status,
           const T* __restrict__ fields,
           long long total_nodes, int interleaved, int frame_velocity, T* __restrict__ out,
           long long* __restrict__ count_out, unsigned long long* __restrict__ stats,
           const unsigned int* __restrict__ tile_hole, DeferQueue dq, int xcd_run) {
  __shared__ double sp[kMaxGrids * 12];
  // the grid table, staged in LDS (dynamic: ngrids records): its fields are
  // read at every candidate grid and walk
  extern __shared__ unsigned long long grid_lds[];
  static_assert(sizeof(GridDev) % 8 == 0, "grid records are staged in 8-byte words");
  for (int i = threadIdx.x; i < ngrids * (int)(sizeof(GridDev) / 8); i += blockDim.x)
    grid_lds[i] = ((const unsigned long long*)grids_g)[i];
  const GridDev* __restrict__ grids = reinterpret_cast<const GridDev*>(grid_lds);
  for (int i = threadIdx.x; i < ngrids * 12; i += blockDim.x) sp[i] = poses[i];
  const int lane = threadIdx.x & 63;
  constexpr int kWaves = BS / 64;
  // this wavefront's rank among the launch's: with xcd_run > 0 the blocks of
  // one XCD take runs of consecutive chunks, whose queries are neighbours on
  // the grids and share donor-cell lines in that XCD's L2
  const long long wrank = xcd_rank(blockIdx.x, gridDim.x, xcd_run) * kWaves + (threadIdx.x >> 6);
  const long long nwaves = (long long)gridDim.x * kWaves;
  // the ids of this lane's query in the wavefront's next chunk, loaded one
  // chunk ahead (the first before the count is known: entries up to the
  // capacity are allocated), so that a chunk starts with them in registers
  int cur_A = 0, cur_m = 0;
  if (wrank * 64 + lane < cap) {
    cur_A = q_grid[wrank * 64 + lane];
    cur_m = q_node[wrank * 64 + lane];
  }
  const unsigned int stamp = *warm.stamp;
  const uint8_t now = (uint8_t)stamp;
  const long long n = min(*d_count, cap);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (count_out) *count_out = *d_count;
    atomicAdd(&stat_slot(stats)[OV_STAT_BACK_CALLS], 1ULL);
    dq.count[(stamp & 1u) ^ 1u] = 0u;  // the other step's counter (its reader is done)
    if (dq.chunk) dq.chunk[(stamp & 1u) ^ 1u] = 0u;
  }
  unsigned int* const dq_count = dq.count + (stamp & 1u);
  unsigned int* const chunk_head = dq.chunk ? dq.chunk + (stamp & 1u) : nullptr;
  __syncthreads();  // the staging is complete
  int my_iters = 0, my_cands = 0;  // this lane's share of the work (walk cells: `visited` of its queries)
  unsigned int my_cells = 0;
  for (long long base = wrank * 64; base < n;) {
    // the wavefront's next chunk (work queue: its ticket, in flight during
    // this chunk)
    unsigned int ticket = 0;
    if (chunk_head && lane == 0) ticket = atomicAdd(chunk_head, 1u);
    const long long q = base + lane;
    const bool mine = q < n;
    int res_grid = -1, res_cell = -1, res_status = OV_Q_ORPHAN;
    T rs[3] = {(T)NAN, (T)NAN, (T)NAN};
    int visited = 0;
    bool limit = false;
    long long key = 0;
    int my_grid = 0;
    int defer = 0;  // kDeferFix or kDeferScan
    int defer_t = 0, defer_cell = -1;
    if (mine) {
      const int A = cur_A;
      const int qm = cur_m;
      my_grid = A;
      // the warm-start entry, read beside the node's coordinates
      int wg, wcell;
      Start ws;
      warm_read(warm, grids[A].node_off + qm, now, wg, wcell, ws);
      T o[3];
      transform_node<T>(grids[A], sp + 12 * A, qm, o);
      qx[q] = o[0];
      qx[cap + q] = o[1];
      qx[2 * cap + q] = o[2];
      const Query Q = make_query<T>(grids, ngrids, sp, flags, A, qm, (double)o[0], (double)o[1], (double)o[2], false);
      key = Q.key;
      if (!Q.finite) {
        atomicOr(dev_status, OV_DEV_NONFINITE);
      } else {
        for (int t = -2; t < ngrids; ++t) {
          const int B = candidate_at(t, Q.A, Q.first);
          if (B < 0) continue;
          const GridDev& G = grids[B];
          double xi[3];
          if (!to_body(G, sp + 12 * B, Q, xi)) continue;
          int seed = -1;
          if (wg == B && wcell >= 0 && (long long)wcell < G.ncells) seed = wcell;
          // the control cell's seed only when there is no warm seed, or
          // for the second walk after a failed warm one
          int rep = -1;
          if (seed < 0) {
            rep = gp(G.brep)[bin_of(G, xi)];
            if (rep < 0) continue;
          }
          int cell = seed >= 0 ? seed : rep;
          T s[3];
          const uint8_t* fl = flags + G.node_off;
          int r = walk<T>(G, fl, xi, Q.err, cell, s, max_walk, limit, visited, &my_iters, tile_hole, stamp,
                          seed >= 0 ? ws : kCentre);
          if (r == kToScan && seed >= 0) {
            rep = gp(G.brep)[bin_of(G, xi)];
            if (rep >= 0 && rep != seed) {
              cell = rep;
              r = walk<T>(G, fl, xi, Q.err, cell, s, max_walk, limit, visited, &my_iters, tile_hole, stamp);
            }
          }
          if (sizeof(T) == 4 && r == kDoubt) {
            defer = kDeferFix;
            defer_t = t;
            defer_cell = cell;
            rs[0] = s[0];  // the FP32 solve's s: the FP64 correction's start
            rs[1] = s[1];
            rs[2] = s[2];
            break;
          }
          if (r == kFound) {
            res_grid = B;
            res_cell = cell;
            res_status = OV_Q_FOUND;
            rs[0] = s[0];
            rs[1] = s[1];
            rs[2] = s[2];
          } else {
            defer = kDeferScan;
            defer_t = t;
            defer_cell = cell;
          }
          break;
        }
      }
    }
    // the next chunk's base, and its ids (fixed stride; or the ticket, which
    // has long arrived)
    long long nbase = base + nwaves * 64;
    if (chunk_head) nbase = (nwaves + (long long)__shfl((int)ticket, 0, 64)) * 64;
    int nxt_A = 0, nxt_m = 0;
    if (nbase + lane < cap) {
      nxt_A = q_grid[nbase + lane];
      nxt_m = q_node[nbase + lane];
    }
    {
      // the wavefront's deferred queries go to the queue with one atomic
      const unsigned long long dm = __ballot(mine && defer != 0);
      if (dm) {
        unsigned int base_slot = 0;
        const int leader = __ffsll((long long)dm) - 1;
        if (lane == leader) base_slot = atomicAdd(dq_count, (unsigned int)__popcll(dm));
        base_slot = __shfl(base_slot, leader, 64);
        if (mine && defer) {
          const unsigned int rank = __popcll(dm & ((1ull << lane) - 1ull));
          if ((long long)(base_slot + rank) < cap) dq.items[base_slot + rank] = (int32_t)q;
          donor_grid[q] = defer;
          donor_cell[q] = defer_cell;
          status[q] = defer_status(defer_t, visited);
          if (defer == kDeferFix) {
            s_out[q] = rs[0];
            s_out[cap + q] = rs[1];
            s_out[2 * cap + q] = rs[2];
          }
        }
      }
    }
    if (mine) {
      my_cells += visited;
      if (limit) atomicOr(dev_status, OV_DEV_WALK_LIMIT);
      if (!defer)
        finish_query<T>(grids, sp, q, cap, key, my_grid, res_grid, res_cell, res_status, visited, rs, donor_grid,
                        donor_cell, s_out, status, warm, now, fields, total_nodes, interleaved, frame_velocity, out);
    }
    base = nbase;
    cur_A = nxt_A;
    cur_m = nxt_m;
  }
  add_work_counters(stats, my_cells, (unsigned int)my_iters, (unsigned int)my_cands);
}

// The whole back half of a step in one kernel, each wavefront on its own: it
// takes 64 queries at a time, one per lane (by a fixed stride over all the
// launch's wavefronts, or from the work queue): the transform; the walk over
// the candidate grids, with the FP64 correction of an undecided FP32 walk
// done at once by its lane; then the wavefront's deferred queries one at a
// time with all its lanes (the brute-force scans); then each lane writes its
// result and interpolates its fields. No barrier: a wavefront never waits
// for another. Every rule that orders candidates, seeds and deferrals is the
// one of the separate passes, so the results are the same bit for bit.
template <typename T, int BS>
__global__ void __launch_bounds__(BS)
    k_back_wave(const GridDev* __restrict__ grids_g, int ngrids, const double* __restrict__ poses,
                const uint8_t* __restrict__ flags, const int32_t* __restrict__ q_grid,
                const int32_t* __restrict__ q_node, T* __restrict__ qx, const long long* __restrict__ d_count,
                long long cap, int32_t* __restrict__ donor_grid, int32_t* __restrict__ donor_cell,
                T* __restrict__ s_out, int32_t* __restrict__ status, Warm warm, int max_walk,
                int32_t* __restrict__ dev_status, const T* __restrict__ fields, long long total_nodes,
                int interleaved, int frame_velocity, T* __restrict__ out, long long* __restrict__ count_out,
                unsigned long long* __restrict__ stats, const unsigned int* __restrict__ tile_hole, DeferQueue dq,
                int xcd_run) {
  __shared__ double sp[kMaxGrids * 12];
  __shared__ ScanLds S;  // (unused: the wavefront scans need none)
  // the grid table, staged in LDS (dynamic: ngrids records): its fields are
  // read at every candidate grid and walk
  extern __shared__ unsigned long long grid_lds[];
  static_assert(sizeof(GridDev) % 8 == 0, "grid records are staged in 8-byte words");
  for (int i = threadIdx.x; i < ngrids * (int)(sizeof(GridDev) / 8); i += blockDim.x)
    grid_lds[i] = ((const unsigned long long*)grids_g)[i];
  const GridDev* __restrict__ grids = reinterpret_cast<const GridDev*>(grid_lds);
  for (int i = threadIdx.x; i < ngrids * 12; i += blockDim.x) sp[i] = poses[i];
  const int lane = threadIdx.x & 63;
  constexpr int kWaves = BS / 64;
  // this wavefront's rank among the launch's: with xcd_run > 0 the blocks of
  // one XCD take runs of consecutive chunks, whose queries are neighbours on
  // the grids and share donor-cell lines in that XCD's L2
  const long long wrank = xcd_rank(blockIdx.x, gridDim.x, xcd_run) * kWaves + (threadIdx.x >> 6);
  const long long nwaves = (long long)gridDim.x * kWaves;
  // the wavefront's chunks: its first two by rank (fixed stride: rank + i
  // nwaves; work queue: then 2 nwaves + a ticket, each taken two chunks
  // ahead). A chunk's ids are loaded two chunks ahead and its queries' node
  // coordinates, warm records and flags one chunk ahead (the first ones
  // before the count is known: entries up to the capacity are allocated)
  long long base = wrank * 64, base1 = (wrank + nwaves) * 64;
  int cur_A = 0, cur_m = 0, nx_A = 0, nx_m = 0;
  if (base + lane < cap) {
    cur_A = q_grid[base + lane];
    cur_m = q_node[base + lane];
  }
  if (base1 + lane < cap) {
    nx_A = q_grid[base1 + lane];
    nx_m = q_node[base1 + lane];
  }
  const unsigned int stamp = *warm.stamp;
  const uint8_t now = (uint8_t)stamp;
  const long long n = min(*d_count, cap);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (count_out) *count_out = *d_count;
    atomicAdd(&stat_slot(stats)[OV_STAT_BACK_CALLS], 1ULL);
    if (dq.chunk) dq.chunk[(stamp & 1u) ^ 1u] = 0u;  // the other step's head (its reader is done)
  }
  unsigned int* const chunk_head = dq.chunk ? dq.chunk + (stamp & 1u) : nullptr;
  __syncthreads();  // the staging is complete
  NodePre pre;
  if (base + lane < n) node_pre_load(grids[cur_A], warm, flags, cur_m, pre);
  int my_iters = 0, my_cands = 0;  // this lane's share of the work (walk cells: `visited` of its queries)
  unsigned int my_cells = 0;
  while (base < n) {
    // the wavefront's chunk after next (work queue: its ticket, in flight
    // during this chunk)
    unsigned int ticket = 0;
    if (chunk_head && lane == 0) ticket = atomicAdd(chunk_head, 1u);
    const long long q = base + lane;
    const bool mine = q < n;
    int res_grid = -1, res_cell = -1, res_status = OV_Q_ORPHAN;
    T rs[3] = {(T)NAN, (T)NAN, (T)NAN};
    int visited = 0;
    bool limit = false;
    long long key = 0;
    int my_grid = 0;
    int defer_st = 0;
    bool defer = false;
    if (mine) {
      const int A = cur_A;
      const int qm = cur_m;
      my_grid = A;
      // the warm-start entry, the node's coordinates and flag (loaded a
      // chunk ahead)
      int wg, wcell;
      Start ws;
      warm_decode(warm, pre.rec, now, wg, wcell, ws);
      T o[3];
      transform_xyz<T>(sp + 12 * A, pre.x, pre.y, pre.z, o);
      qx[q] = o[0];
      qx[cap + q] = o[1];
      qx[2 * cap + q] = o[2];
      const Query Q = query_from<T>(grids, ngrids, sp, A, qm, (uint8_t)pre.flag, (double)o[0], (double)o[1],
                                    (double)o[2], false, pre.x, pre.y, pre.z);
      key = Q.key;
      if (!Q.finite) {
        atomicOr(dev_status, OV_DEV_NONFINITE);
      } else {
        for (int t = -2; t < ngrids; ++t) {
          const int B = candidate_at(t, Q.A, Q.first);
          if (B < 0) continue;
          const GridDev& G = grids[B];
          double xi[3];
          if (!to_body(G, sp + 12 * B, Q, xi)) continue;
          int seed = -1;
          if (wg == B && wcell >= 0 && (long long)wcell < G.ncells) seed = wcell;
          // the control cell's seed only when there is no warm seed, or
          // for the second walk after a failed warm one
          int rep = -1;
          if (seed < 0) {
            rep = gp(G.brep)[bin_of(G, xi)];
            if (rep < 0) continue;
          }
          int cell = seed >= 0 ? seed : rep;
          T s[3];
          const uint8_t* fl = flags + G.node_off;
          int r = walk<T>(G, fl, xi, Q.err, cell, s, max_walk, limit, visited, &my_iters, tile_hole, stamp,
                          seed >= 0 ? ws : kCentre);
          if (r == kToScan && seed >= 0) {
            rep = gp(G.brep)[bin_of(G, xi)];
            if (rep >= 0 && rep != seed) {
              cell = rep;
              r = walk<T>(G, fl, xi, Q.err, cell, s, max_walk, limit, visited, &my_iters, tile_hole, stamp);
            }
          }
          int how = OV_Q_FOUND;
          if (sizeof(T) == 4 && r == kDoubt) {
            // the FP64 correction: the walk goes on from this cell in FP64
            // on the exact position
            const Query QE = make_query<T>(grids, ngrids, sp, flags, A, Q.m, 0.0, 0.0, 0.0, true);
            double xe[3], s64[3];
            body_frame(sp + 12 * B, QE.x, xe);
            r = walk<double, false>(G, fl, xe, 0.0, cell, s64, max_walk, limit, visited, &my_iters, nullptr, 0u,
                                    start_from<T>(s));
            s[0] = (T)s64[0];
            s[1] = (T)s64[1];
            s[2] = (T)s64[2];
            how = OV_Q_FOUND | OV_Q_FP64_FIXED;
          }
          if (r == kFound) {
            res_grid = B;
            res_cell = cell;
            res_status = how;
            rs[0] = s[0];
            rs[1] = s[1];
            rs[2] = s[2];
          } else {
            defer = true;
            defer_st = defer_status(t, visited);
          }
          break;
        }
      }
    }
    // the chunk after next, and its ids (fixed stride; or the ticket, which
    // has long arrived); the next chunk's node data, in flight during the
    // scans and the finish of this one
    long long base2 = base1 + nwaves * 64;
    if (chunk_head) base2 = (2 * nwaves + (long long)__shfl((int)ticket, 0, 64)) * 64;
    int nxt_A = 0, nxt_m = 0;
    if (base2 + lane < cap) {
      nxt_A = q_grid[base2 + lane];
      nxt_m = q_node[base2 + lane];
    }
    NodePre pre1;
    if (base1 + lane < n) node_pre_load(grids[nx_A], warm, flags, nx_m, pre1);
    // the wavefront's deferred queries, one at a time with all its lanes
    for (unsigned long long dm = __ballot(defer); dm; dm &= dm - 1) {
      const int owner = __ffsll((long long)dm) - 1;
      int g_grid, g_cell, g_status, dvisited, walk_iters = 0;  // (walk work counted once, by the owner)
      T gs[3];
      bool dlimit = false;
      deferred_scan_one<T, true>(grids, ngrids, sp, flags, __shfl(cur_A, owner, 64), __shfl(cur_m, owner, 64),
                                 __shfl(defer_st, owner, 64), S, max_walk, g_grid, g_cell, g_status, gs, dvisited,
                                 dlimit, walk_iters, my_iters, my_cands);
      if (lane == owner) {
        res_grid = g_grid;
        res_cell = g_cell;
        res_status = g_status;
        rs[0] = gs[0];
        rs[1] = gs[1];
        rs[2] = gs[2];
        visited = dvisited;
        limit |= dlimit;
        my_iters += walk_iters;
      }
    }
    if (mine) {
      my_cells += visited;
      if (limit) atomicOr(dev_status, OV_DEV_WALK_LIMIT);
      finish_query<T>(grids, sp, q, cap, key, my_grid, res_grid, res_cell, res_status, visited, rs, donor_grid,
                      donor_cell, s_out, status, warm, now, fields, total_nodes, interleaved, frame_velocity, out);
    }
    base = base1;
    base1 = base2;
    cur_A = nx_A;
    cur_m = nx_m;
    nx_A = nxt_A;
    nx_m = nxt_m;
    pre = pre1;
  }
  add_work_counters(stats, my_cells, (unsigned int)my_iters, (unsigned int)my_cands);
}

// The second kernel of the two-kernel back half: the queued queries of this
// step (stamp parity), BS per block at a time, one per thread: the FP64
// correction of an undecided FP32 walk (the walk goes on in FP64 from its
// cell, on the exact position); then the block's queries still without a
// donor one at a time with all its threads (the cooperative scans); then
// each thread writes its result and interpolates. The work counters add the
// cells, iterations and candidates of this kernel only.
template <typename T, int BS>
__global__ void __launch_bounds__(BS)
    k_back_defer(const GridDev* __restrict__ grids_g, int ngrids, const double* __restrict__ poses,
                 const uint8_t* __restrict__ flags, const int32_t* __restrict__ q_grid,
                 const int32_t* __restrict__ q_node, long long cap, int32_t* __restrict__ donor_grid,
                 int32_t* __restrict__ donor_cell, T* __restrict__ s_out, int32_t* __restrict__ status, Warm warm,
                 int max_walk, int32_t* __restrict__ dev_status, const T* __restrict__ fields, long long total_nodes,
                 int interleaved, int frame_velocity, T* __restrict__ out, unsigned long long* __restrict__ stats,
                 DeferQueue dq) {
  __shared__ double sp[kMaxGrids * 12];
  __shared__ int list_owner[BS], list_st[BS];
  __shared__ long long list_q[BS];
  __shared__ int nlist;
  __shared__ ScanLds S;
  extern __shared__ unsigned long long grid_lds[];
  const unsigned int stamp = *warm.stamp;
  const uint8_t now = (uint8_t)stamp;
  const long long n = min((long long)dq.count[stamp & 1u], cap);
  // entry i goes to block i mod gridDim.x: the usual few queued queries
  // (each a chain of FP64 Newton solves, or a block-wide scan) spread over
  // the blocks instead of queueing in one
  if ((long long)blockIdx.x >= n) return;  // nothing for this block (same in every thread)
  for (int i = threadIdx.x; i < ngrids * (int)(sizeof(GridDev) / 8); i += blockDim.x)
    grid_lds[i] = ((const unsigned long long*)grids_g)[i];
  const GridDev* __restrict__ grids = reinterpret_cast<const GridDev*>(grid_lds);
  for (int i = threadIdx.x; i < ngrids * 12; i += blockDim.x) sp[i] = poses[i];
  int my_iters = 0, my_cands = 0;
  unsigned int my_cells = 0;
  for (long long base = 0; base + blockIdx.x < n; base += (long long)gridDim.x * blockDim.x) {
    if (threadIdx.x == 0) nlist = 0;
    __syncthreads();
    const long long idx = base + (long long)threadIdx.x * gridDim.x + blockIdx.x;
    const bool mine = idx < n;
    long long q = 0, key = 0;
    int my_grid = 0, visited = 0, visited0 = 0;
    int res_grid = -1, res_cell = -1, res_status = OV_Q_ORPHAN;
    T rs[3] = {(T)NAN, (T)NAN, (T)NAN};
    bool limit = false;
    if (mine) {
      q = dq.items[idx];
      const int marker = donor_grid[q];
      int cell = donor_cell[q];
      const int st = status[q];
      const int t0 = (st & 255) - 2;
      visited = visited0 = (st >> 8) & 255;
      const int A = q_grid[q];
      my_grid = A;
      const Query QE = make_query<T>(grids, ngrids, sp, flags, A, q_node[q], 0.0, 0.0, 0.0, true);
      key = QE.key;
      bool scan = true;
      if (sizeof(T) == 4 && marker == kDeferFix) {
        const int B = candidate_at(t0, A, QE.first);
        const GridDev& G = grids[B];
        double xe[3], s64[3];
        body_frame(sp + 12 * B, QE.x, xe);
        const T sq[3] = {s_out[q], s_out[cap + q], s_out[2 * cap + q]};
        const int r = walk<double, false>(G, flags + G.node_off, xe, 0.0, cell, s64, max_walk, limit, visited,
                                          &my_iters, nullptr, 0u, start_from<T>(sq));
        if (r == kFound) {
          res_grid = B;
          res_cell = cell;
          res_status = OV_Q_FOUND | OV_Q_FP64_FIXED;
          rs[0] = (T)s64[0];
          rs[1] = (T)s64[1];
          rs[2] = (T)s64[2];
          scan = false;
        }
      }
      if (scan) {
        const int slot = atomicAdd(&nlist, 1);
        list_owner[slot] = (int)threadIdx.x;
        list_q[slot] = q;
        list_st[slot] = defer_status(t0, visited);
      }
    }
    __syncthreads();
    block_deferred_scans<T>(grids, ngrids, sp, flags, q_grid, q_node, nlist, list_owner, list_q, list_st, S, max_walk,
                            res_grid, res_cell, res_status, rs, visited, limit, my_iters, my_cands);
    if (mine) {
      my_cells += (unsigned int)max(0, visited - visited0);
      if (limit) atomicOr(dev_status, OV_DEV_WALK_LIMIT);
      finish_query<T>(grids, sp, q, cap, key, my_grid, res_grid, res_cell, res_status, visited, rs, donor_grid,
                      donor_cell, s_out, status, warm, now, fields, total_nodes, interleaved, frame_velocity, out);
    }
    __syncthreads();  // nlist and the list are rebuilt for the next range
  }
  add_work_counters(stats, my_cells, (unsigned int)my_iters, (unsigned int)my_cands);
}

static Warm warm_of(ov_ctx* ctx, int slot) {
  return Warm{ctx->d_warm, ctx->d_stamp + 1 + slot, ctx->warm};
}

template <typename T>
static void launch_search_t(ov_ctx* ctx, const double* poses, const uint8_t* flags, const int32_t* q_grid,
                            const int32_t* q_node, const T* qx, const long long* d_count, long long capacity,
                            int32_t* donor_grid, int32_t* donor_cell, T* s, int32_t* status, hipStream_t st,
                            int slot) {
  const Warm warm = warm_of(ctx, slot);
  const int ng = (int)ctx->grids.size();
  const int block = ctx->search_block;
  long long grid = grid_size_for(ctx, capacity, block);
  hipLaunchKernelGGL(k_donor_walk<T>, dim3((unsigned)grid), dim3(block), 0, st, ctx->d_grids, ng, poses, flags,
                     q_grid, q_node, qx, d_count, capacity, donor_grid, donor_cell, s, status, warm, ctx->max_walk,
                     ctx->d_status);
  // the sweeps: one lane (FP64 correction) or one block per 256 queries (scan)
  const long long sweep_cap = (long long)ctx->num_cus * 8;
  if (sizeof(T) == 4)
    hipLaunchKernelGGL(k_donor_fix, dim3((unsigned)std::max(1LL, std::min(sweep_cap, (capacity + 255) / 256))),
                       dim3(256), 0, st, ctx->d_grids, ng, poses, flags, q_grid, q_node, (const float*)qx, d_count,
                       capacity, donor_grid, donor_cell, (float*)s, status, warm,
                       ctx->max_walk, ctx->d_status);
  hipLaunchKernelGGL(k_donor_scan<T>, dim3((unsigned)std::max(1LL, std::min(sweep_cap, (capacity + 255) / 256))),
                     dim3(256), 0, st, ctx->d_grids, ng, poses, flags, q_grid, q_node, qx, d_count, capacity,
                     donor_grid, donor_cell, s, status, warm, ctx->max_walk,
                     ctx->d_status);
}

template <typename T>
static void launch_back_t(ov_ctx* ctx, const double* poses, const uint8_t* flags, const int32_t* q_grid,
                          const int32_t* q_node, T* qx, const long long* d_count, long long capacity,
                          int32_t* donor_grid, int32_t* donor_cell, T* s, int32_t* status, const T* fields,
                          T* out, long long* count_out, hipStream_t st, int slot, const DeferQueue* dq) {
  const Warm warm = warm_of(ctx, slot);
  const int bs = ctx->back_block;
  const long long grid =
      std::max(1LL, std::min((long long)ctx->num_cus * ctx->back_blocks_per_cu, (capacity + bs - 1) / bs));
  const bool split = dq != nullptr && dq->items != nullptr;
  const DeferQueue q = dq ? *dq : DeferQueue{nullptr, nullptr, nullptr};
#define OV_BACK_ARGS                                                                                             \
  ctx->d_grids, (int)ctx->grids.size(), poses, flags, q_grid, q_node, qx, d_count, capacity, donor_grid, donor_cell, \
      s, status, warm, ctx->max_walk, ctx->d_status, fields,                                                       \
      ctx->node_off.back(), ctx->field_layout, ctx->frame_velocity, out, count_out, ctx->d_stats,                  \
      ctx->d_tile_hole + slot * std::max(1LL, ctx->total_tiles), q, ctx->back_xcd
#define OV_DEFER_ARGS                                                                                            \
  ctx->d_grids, (int)ctx->grids.size(), poses, flags, q_grid, q_node, capacity, donor_grid, donor_cell, s, status, \
      warm, ctx->max_walk, ctx->d_status, fields, ctx->node_off.back(), ctx->field_layout, ctx->frame_velocity, out, \
      ctx->d_stats, q
  const size_t lds = sizeof(GridDev) * ctx->grids.size();
  const dim3 g((unsigned)grid);
  if (!split) {
    if (bs == 64) hipLaunchKernelGGL((k_back_wave<T, 64>), g, dim3(64), lds, st, OV_BACK_ARGS);
    else if (bs == 128) hipLaunchKernelGGL((k_back_wave<T, 128>), g, dim3(128), lds, st, OV_BACK_ARGS);
    else hipLaunchKernelGGL((k_back_wave<T, 256>), g, dim3(256), lds, st, OV_BACK_ARGS);
  } else {
    // the second kernel: usually a few queries; as many blocks as CUs
    const dim3 gd((unsigned)std::max(1LL, std::min((long long)ctx->num_cus, (capacity + bs - 1) / bs)));
    if (bs == 64) {
      hipLaunchKernelGGL((k_back_walk<T, 64>), g, dim3(64), lds, st, OV_BACK_ARGS);
      hipLaunchKernelGGL((k_back_defer<T, 64>), gd, dim3(64), lds, st, OV_DEFER_ARGS);
    } else if (bs == 128) {
      hipLaunchKernelGGL((k_back_walk<T, 128>), g, dim3(128), lds, st, OV_BACK_ARGS);
      hipLaunchKernelGGL((k_back_defer<T, 128>), gd, dim3(128), lds, st, OV_DEFER_ARGS);
    } else {
      hipLaunchKernelGGL((k_back_walk<T, 256>), g, dim3(256), lds, st, OV_BACK_ARGS);
      hipLaunchKernelGGL((k_back_defer<T, 256>), gd, dim3(256), lds, st, OV_DEFER_ARGS);
    }
  }
#undef OV_BACK_ARGS
#undef OV_DEFER_ARGS
}

hipError_t launch_donor_search(ov_ctx* ctx, const double* poses, const uint8_t* flags, const int32_t* q_grid,
                               const int32_t* q_node, const void* qx, const long long* d_count, long long capacity,
                               int32_t* donor_grid, int32_t* donor_cell, void* s, int32_t* status, hipStream_t st,
                               int slot) {
  if (ctx->precision == OV_MIXED)
    launch_search_t<float>(ctx, poses, flags, q_grid, q_node, (const float*)qx, d_count, capacity, donor_grid,
                           donor_cell, (float*)s, status, st, slot);
  else
    launch_search_t<double>(ctx, poses, flags, q_grid, q_node, (const double*)qx, d_count, capacity, donor_grid,
                            donor_cell, (double*)s, status, st, slot);
  return hipGetLastError();
}

__global__ void k_copy_count(long long* __restrict__ dst, const long long* __restrict__ src) { *dst = *src; }

hipError_t launch_copy_count(long long* dst, const int64_t* src, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, st, dst, (const long long*)src);
  return hipGetLastError();
}

hipError_t launch_back(ov_ctx* ctx, const double* poses, const uint8_t* flags, const int32_t* q_grid,
                       const int32_t* q_node, void* qx, const long long* d_count, long long capacity,
                       int32_t* donor_grid, int32_t* donor_cell, void* s, int32_t* status, const void* fields,
                       void* out, long long* count_out, hipStream_t st, int slot, int32_t* defer_items,
                       unsigned int* defer_count) {
  if (capacity > 0 && ctx->back_fused) {
    // defer_count: [0, 2) the deferral queue's counters, [2, 4) the work queue's heads
    const bool split = ctx->back_fused == 2 && defer_items && defer_count;
    const bool queue = ctx->back_queue && defer_count;
    DeferQueue dq{split ? defer_items : nullptr, split ? defer_count : nullptr, queue ? defer_count + 2 : nullptr};
    const DeferQueue* q = (split || queue) ? &dq : nullptr;
    if (ctx->precision == OV_MIXED)
      launch_back_t<float>(ctx, poses, flags, q_grid, q_node, (float*)qx, d_count, capacity, donor_grid, donor_cell,
                           (float*)s, status, (const float*)fields, (float*)out, count_out, st, slot, q);
    else
      launch_back_t<double>(ctx, poses, flags, q_grid, q_node, (double*)qx, d_count, capacity, donor_grid,
                            donor_cell, (double*)s, status, (const double*)fields, (double*)out, count_out, st,
                            slot, q);
    return hipGetLastError();
  }
  hipError_t e = hipSuccess;
  if (capacity > 0) {
    e = launch_transform(ctx, poses, q_grid, q_node, d_count, capacity, qx, st);
    if (e == hipSuccess)
      e = launch_donor_search(ctx, poses, flags, q_grid, q_node, qx, d_count, capacity, donor_grid, donor_cell, s,
                              status, st, slot);
    if (e == hipSuccess && fields)
      e = launch_interp(ctx, donor_grid, donor_cell, s, d_count, capacity, fields, out, st);
    if (e == hipSuccess && fields && ctx->frame_velocity)
      e = launch_frame_velocity(ctx, poses, q_grid, donor_grid, d_count, capacity, out, st);
  }
  if (e == hipSuccess && count_out) e = launch_copy_count(count_out, (const int64_t*)d_count, st);
  return e;
}

}  // namespace ov

using namespace ov;

extern "C" int overset_donor_search(ov_ctx* ctx, const double* poses, const uint8_t* flags, const int32_t* q_grid,
                                    const int32_t* q_node, const void* qx, const int64_t* d_count, int64_t capacity,
                                    int32_t* donor_grid, int32_t* donor_cell, void* s, int32_t* status,
                                    void* stream) {
  if (!ctx) return OV_EINVAL;
  if (!ctx->finalized) return fail(ctx, OV_ESTATE, "step call before ov_finalize");
  if (capacity < 0) return fail(ctx, OV_EINVAL, "overset_donor_search: negative capacity");
  if (capacity == 0) return OV_OK;
  if (!poses || !flags || !q_grid || !q_node || !qx || !d_count || !donor_grid || !donor_cell || !s || !status)
    return fail(ctx, OV_EINVAL, "overset_donor_search: null pointer");
  hipError_t e = launch_donor_search(ctx, poses, flags, q_grid, q_node, qx, (const long long*)d_count, capacity,
                                     donor_grid, donor_cell, s, status, (hipStream_t)stream, 0);
  return e == hipSuccess ? OV_OK : hip_fail(ctx, e, "overset_donor_search");
}
