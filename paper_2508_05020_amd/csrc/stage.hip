// The fused stage kernel of libamr for gfx950 (CDNA4, wave64): per (patch,
// tile) work item, primitives of the tile and its halos in LDS, WENO5-JS
// interpolation and the Rusanov flux at every edge (Eq. (10)-(12)), the
// face fluxes and divergence of Eq. (9) in flux form, and the SSP-RK3 stage
// combination; also the tile variants the autotuner chooses from.
//
// Floating-point contract: implicit contraction is off and every fused
// multiply-add is written with fma(), so a cell's operation sequence is fixed
// by this source and identical for every tile variant, fused or explicit
// halo, per-patch or batched launch.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "amr_internal.hpp"

// no implicit contraction anywhere in this file
#pragma clang fp contract(off)

#include "device_common.hpp"

namespace amr {
namespace {

// ---------------------------------------------------------------------------
// fused right-hand side + SSP-RK3 stage on (pid, tile) work items
// ---------------------------------------------------------------------------

// threadIdx.x hidden from the optimiser: the index arithmetic of a phase is
// then formed in that phase instead of being shared with another direction's
// phase and held in registers across the edge phases, where they run out
__device__ __forceinline__ int phase_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (relative error near one ulp); used where correct rounding is not required.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(x) for x > 0 from the hardware reciprocal square-root estimate
// (relative error near 2^-24): one coupled Goldschmidt step for sqrt(x) and
// 1/(2 sqrt(x)), then one Newton correction of the root (a few ulp).  Used
// for the sound speed in the Rusanov dissipation only.
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}

// sqrt(x) and 1/sqrt(x) for x > 0 from the hardware reciprocal square-root
// estimate: two coupled Goldschmidt steps for sqrt(x) and 1/(2 sqrt(x)),
// then one Newton correction of the root (both within a few ulp).
__device__ __forceinline__ void sqrt_rsqrt_nr(double x, double& s, double& is) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  s = fma(fma(-g, g, x), h, g);
  is = 2.0 * h;
}

// Numerator and denominator of the nonlinear WENO5-JS combination of three
// candidates q_k from e_k = eps + b_k (b_k the smoothness indicators): the
// value is sum(alpha_k q_k) / sum(alpha_k) with alpha_k = d_k / t_k, t_k =
// e_k^2 and d = (1, 10, 5)/16, evaluated as cross products (alpha_k times
// t0 t1 t2 / 16): num = t2 (t1 q0 + 10 t0 q1) + 5 t0 t1 q2, den = t2 (t1 +
// 10 t0) + 5 t0 t1.
__device__ __forceinline__ void weno_num_den(double e0, double e1, double e2, double q0, double q1,
                                             double q2, double& num, double& den) {
  const double t0 = e0 * e0, t1 = e1 * e1, t2 = e2 * e2;
  const double c0 = 10.0 * t0;
  const double p5 = 5.0 * (t0 * t1);
  den = fma(t2, c0 + t1, p5);
  num = fma(t2, fma(c0, q1, t1 * q0), p5 * q2);
}

// WENO5-JS point values on both sides of the edge between v2 and v3 from the
// six nodes v0..v5: the left-biased value from v0..v4 and the right-biased
// value from the mirrored stencil v5..v1.  Candidates: the quadratic through
// three consecutive nodes evaluated at the edge (x8), two of which the sides
// share.  Indicators (x4): 13/12 k^2 + 1/4 s^2 of the Jiang-Shu definition
// for the window (a, b, c), with k = a - 2b + c and s the first-derivative
// form at the node the edge adjoins: a - 4b + 3c (window left of the edge),
// a - c (centred), 3a - 4b + c (window right of it).  With the first
// differences d_i = v_(i+1) - v_i, k_w = d_(w+1) - d_w and the three forms
// are k + 2 d_(w+1), -(d_w + d_(w+1)) and k - 2 d_w, so the four windows
// share their differences.  The curvature term of a window (with eps) is
// shared by the two sides where both use the window.  One reciprocal serves
// both sides: 1/(den_L den_R) (the indicators are bounded below by eps, and
// eps is at least 1e-20, so the product stays a normal number) times the
// other side's denominator, and with it the final 1/8.  The scalings are
// powers of two.
__device__ __forceinline__ void weno5_pair(double v0, double v1, double v2, double v3, double v4,
                                           double v5, double eps4, double& L, double& R) {
  const double qa = fma(15.0, v2, fma(-10.0, v1, 3.0 * v0));  // left, nodes v0..v2
  const double qb = fma(3.0, v3, fma(6.0, v2, -v1));          // nodes v1..v3 (both sides)
  const double qc = fma(6.0, v3, fma(3.0, v2, -v4));          // nodes v2..v4 (both sides)
  const double qd = fma(15.0, v3, fma(-10.0, v4, 3.0 * v5));  // right, nodes v3..v5
  const double d0 = v1 - v0, d1 = v2 - v1, d2 = v3 - v2, d3 = v4 - v3, d4 = v5 - v4;
  const double k0 = d1 - d0, k1 = d2 - d1, k2 = d3 - d2, k3 = d4 - d3;
  constexpr double c4 = 4.0 * (13.0 / 12.0);
  // eps + curvature term of windows v0..v2, v1..v3, v2..v4, v3..v5
  const double h0 = fma(c4 * k0, k0, eps4);
  const double h1 = fma(c4 * k1, k1, eps4);
  const double h2 = fma(c4 * k2, k2, eps4);
  const double h3 = fma(c4 * k3, k3, eps4);
  const double sl0 = fma(2.0, d1, k0);   // window v0..v2, node v2
  const double sl1 = d1 + d2;            // window v1..v3, centred
  const double sl2 = fma(-2.0, d2, k2);  // window v2..v4, node v2
  const double sr0 = fma(-2.0, d3, k3);  // window v3..v5, node v3
  const double sr1 = d2 + d3;            // window v2..v4, centred
  const double sr2 = fma(2.0, d2, k1);   // window v1..v3, node v3
  double nl, dl, nr, dr;
  weno_num_den(fma(sl0, sl0, h0), fma(sl1, sl1, h1), fma(sl2, sl2, h2), qa, qb, qc, nl, dl);
  weno_num_den(fma(sr0, sr0, h3), fma(sr1, sr1, h2), fma(sr2, sr2, h1), qd, qc, qb, nr, dr);
  const double inv = rcp_nr(dl * dr) * 0.125;
  L = nl * (dr * inv);
  R = nr * (dl * inv);
}

__device__ __forceinline__ double central4(double b, double c, double d, double e) {
  return fma(9.0, c + d, -(b + e)) * 0.0625;
}

template <int D>
struct EdgeState {
  double p, T, u[D];
};

// Density, total energy and direction-J signal speed |u_J| + c of an edge
// state (Eq. (5)-(7), T = p / rho).
template <int D, int J>
__device__ __forceinline__ void edge_thermo(const DevMesh& m, const EdgeState<D>& w, double& rho,
                                            double& E, double& speed) {
  rho = w.p * rcp_nr(w.T);
  double uu = w.u[0] * w.u[0];
#pragma unroll
  for (int i = 1; i < D; ++i) uu = fma(w.u[i], w.u[i], uu);
  E = fma(0.5 * rho, uu, w.p * m.igm1);
  speed = sqrt_nr(m.gamma * w.T) + fabs(w.u[J]);
}

// Variable v of the conserved state and of the direction-J flux of an edge
// state (Eq. (1)-(3)).
template <int D, int J>
__device__ __forceinline__ void edge_uf(const EdgeState<D>& w, double rho, double E, int v,
                                        double& U, double& F) {
  if (v == 0) {
    U = rho;
    F = rho * w.u[J];
  } else if (v == D + 1) {
    U = E;
    F = (E + w.p) * w.u[J];
  } else {
    const int i = v - 1;
    double ui = w.u[0];
#pragma unroll
    for (int k = 1; k < D; ++k)
      if (k == i) ui = w.u[k];
    const double mi = rho * ui;
    U = mi;
    F = (i == J) ? fma(mi, w.u[J], w.p) : mi * w.u[J];
  }
}

template <int D, int TX, int TY, int TZ>
struct TileShape {
  static constexpr int T0 = TX;
  static constexpr int T1 = D >= 2 ? TY : 1;
  static constexpr int T2 = D >= 3 ? TZ : 1;
  static constexpr int NCELL = T0 * T1 * T2;
  // Row pitch (doubles) of the node arrays in LDS: the union box of 1D/2D
  // tiles and the x-extended box of 3D tiles have rows of T0 + 8 nodes, a
  // multiple of 8 for the tile widths used; an odd pitch starts successive
  // rows in different banks, so the lanes of a wave that read or write
  // neighbouring rows do not collide.  The y- and z-extended 3D boxes are
  // read in runs of whole rows and keep their width.
  static constexpr int UPITCH = D == 1 ? T0 + 8 : ((T0 + 8) | 1);
  static constexpr int NUNION = UPITCH * (D >= 2 ? T1 + 8 : 1);
  static constexpr int xpitch(int j) { return j == 0 ? ((T0 + 8) | 1) : T0; }
  static constexpr int ext(int j) {
    return xpitch(j) * (T1 + (j == 1 ? 8 : 0)) * (T2 + (j == 2 ? 8 : 0));
  }
  static constexpr int edges(int j) {
    return (T0 + (j == 0 ? 3 : 0)) * (T1 + (j == 1 ? 3 : 0)) * (T2 + (j == 2 ? 3 : 0));
  }
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int EXTMAX = cmax(ext(0), cmax(D >= 2 ? ext(1) : 0, D >= 3 ? ext(2) : 0));
  static constexpr int EDMAX =
      cmax(edges(0), cmax(D >= 2 ? edges(1) : 0, D >= 3 ? edges(2) : 0));
};

// Primitives (p, T, u_j) of one node from its conserved values.
template <int D>
__device__ __forceinline__ void node_primitives(const DevMesh& m, const double* u, double* q) {
  const double r = rcp_nr(u[0]);
  double ke = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double ui = u[1 + i] * r;
    ke = (i == 0) ? u[1] * ui : fma(u[1 + i], ui, ke);
    q[2 + i] = ui;
  }
  const double p = m.gm1 * fma(-0.5, ke, u[D + 1]);
  q[0] = p;
  q[1] = p * r;
}

// What the edge phase reads of a node: its primitives (p, T, u_j), or for
// the characteristic scheme its conserved values, at sP[k NEXT + idx].
template <int D, bool CHAR>
__device__ __forceinline__ void node_store(const DevMesh& m, const double* u, double* sP, int next,
                                           int idx) {
  if constexpr (CHAR) {
#pragma unroll
    for (int v = 0; v < D + 2; ++v) sP[v * next + idx] = u[v];
  } else {
    double q[D + 2];
    node_primitives<D>(m, u, q);
#pragma unroll
    for (int k = 0; k < D + 2; ++k) sP[k * next + idx] = q[k];
  }
}


// Same-level patches around the tile's patch, by offset code
// (o0+1) + 3 (o1+1) + 9 (o2+1), o in {-1,0,1}^D (periodic wrap), as the
// offsets of their data in the state buffer (-1 where no patch or outside a
// non-periodic domain), looked up once per block.
template <int D>
__device__ __forceinline__ void load_neighbours(const DevMesh& m, int l, const int pc[3],
                                                long long* sNB) {
  constexpr int NO = D == 1 ? 3 : (D == 2 ? 9 : 27);
  const int t = threadIdx.x;
  if (t < NO) {
    const int np = m.lv[l].np;
    int q[3] = {0, 0, 0};
    bool in = true;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int o = (j == 0 ? t : (j == 1 ? t / 3 : t / 9)) % 3 - 1;
      int v = pc[j] + o;
      if (v < 0 || v >= np) {
        if (m.periodic[j]) v = (v + np) % np;
        else in = false;
      }
      q[j] = v;
    }
    const int pid = in ? map_at<D>(m, l, q) : -1;
    sNB[t] = pid >= 0 ? patch_base(m, pid, l) : -1;
  }
}

// Conserved values of a node at patch-local cell c (may lie in the halo,
// at most 4 cells outside the patch): from the patch itself, or by the
// ghost-fill rule when outside the patch (same-level source from the
// neighbour table, where a position beyond a transmissive boundary is the
// nearest cell of this patch, else the patch's own ghost layer, which holds
// the prolonged value).
template <int D, bool FUSE>
__device__ __forceinline__ void node_conserved(const DevMesh& m, const double* __restrict__ Uin,
                                               const double* __restrict__ Pin, int n, int full,
                                               const int c[3], const int pc[3], int l,
                                               const long long* sNB, double* u) {
  constexpr int NV = D + 2;
  bool inside = true;
  for (int j = 0; j < D; ++j) inside &= (c[j] >= 0 && c[j] < n);
  const int vs = var_stride<D>(full);
  if (FUSE && !inside) {
    const int np = m.lv[l].np;
    int code = 0, loc[3] = {0, 0, 0}, mul = 1;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      int o = c[j] < 0 ? -1 : (c[j] >= n ? 1 : 0);
      int lj = o == 0 ? c[j] : (o < 0 ? c[j] + n : c[j] - n);
      if (o != 0 && !m.periodic[j] && (unsigned)(pc[j] + o) >= (unsigned)np) {
        o = 0;
        lj = c[j] < 0 ? 0 : n - 1;
      }
      loc[j] = lj;
      code += (o + 1) * mul;
      mul *= 3;
    }
    const long long sb = sNB[code];
    if (sb >= 0) {
      const double* S = Uin + sb;
      const int off = box_off<D>(full, loc[0] + NG, loc[1] + NG, loc[2] + NG);
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = S[v * vs + off];
      return;
    }
    // no same-level source: the prolonged ghost value was written into the
    // patch's own ghost layer by the coarse-ghost fill pass
  }
  const int off = box_off<D>(full, c[0] + NG, c[1] + NG, c[2] + NG);
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = Pin[v * vs + off];
}

// node_conserved for a node of a 3D tile's halo along J (or of the tile
// itself): only its J component can lie outside the patch, so the neighbour
// code and the wrap or clamp are formed for that component alone.
template <int D, int J, bool FUSE>
__device__ __forceinline__ void node_conserved_dir(const DevMesh& m,
                                                   const double* __restrict__ Uin,
                                                   const double* __restrict__ Pin, int n,
                                                   int full, const int c[3], const int pc[3],
                                                   int l, const long long* sNB, double* u) {
  constexpr int NV = D + 2;
  constexpr int CENTRE = D == 1 ? 1 : (D == 2 ? 4 : 13);
  constexpr int MULJ = J == 0 ? 1 : (J == 1 ? 3 : 9);
  const int vs = var_stride<D>(full);
  const double* src = Pin;
  int cj = c[J];
  if (FUSE && (unsigned)cj >= (unsigned)n) {
    int o = cj < 0 ? -1 : 1;
    int lj = cj < 0 ? cj + n : cj - n;
    if (!m.periodic[J] && (unsigned)(pc[J] + o) >= (unsigned)m.lv[l].np) {
      o = 0;
      lj = cj < 0 ? 0 : n - 1;
    }
    const long long sb = sNB[CENTRE + o * MULJ];
    // no same-level source: the prolonged ghost value in the patch's own
    // ghost layer (position unchanged)
    if (sb >= 0) {
      src = Uin + sb;
      cj = lj;
    }
  }
  const int off = box_off<D>(full, (J == 0 ? cj : c[0]) + NG, (J == 1 ? cj : c[1]) + NG,
                             (J == 2 ? cj : c[2]) + NG);
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = src[v * vs + off];
}

// 1D/2D: primitives of the tile plus 4-node halos in every direction
// (corner nodes, used by no stencil, are skipped), loaded once per launch.
template <int D, int TX, int TY, int NT, bool FUSE, bool CHAR>
__device__ __forceinline__ void load_union(const DevMesh& m, const double* __restrict__ Uin,
                                           const double* __restrict__ Pin, int n, int full,
                                           const int o[3], const int pc[3], int l,
                                           const long long* sN, double* sP) {
  using S = TileShape<D, TX, TY, 1>;
  constexpr int T0 = TX, T1 = D >= 2 ? TY : 1;
  constexpr int U0 = T0 + 8, U1 = D >= 2 ? T1 + 8 : 1;
  constexpr int NU = U0 * U1;
  for (int idx = threadIdx.x; idx < NU; idx += NT) {
    const int e0 = idx % U0, e1 = idx / U0;
    const bool hx = e0 < 4 || e0 >= T0 + 4;
    const bool hy = D >= 2 && (e1 < 4 || e1 >= T1 + 4);
    if (hx && hy) continue;
    const int c[3] = {o[0] + e0 - 4, D >= 2 ? o[1] + e1 - 4 : 0, 0};
    double u[D + 2];
    node_conserved<D, FUSE>(m, Uin, Pin, n, full, c, pc, l, sN, u);
    node_store<D, CHAR>(m, u, sP, S::NUNION, e0 + S::UPITCH * e1);
  }
}

// Riemann flux of direction J at one edge whose window (nodes i-2 .. i+3)
// starts at layout index `base` of the primitives in LDS (NEXT nodes per
// primitive, STEP between neighbours along J); stored doubled at sF[v NED + e].
template <int D, int J, int NEXT, int STEP, int NED, bool CENTRAL>
__device__ __forceinline__ void edge_at_scheme(const DevMesh& m, const double* sP, int base,
                                               double* sF, int e) {
  constexpr int NV = D + 2;
  const double eps4 = 4.0 * m.eps;
  // interpolated left/right values of primitive q (p, T, u_j) at this edge,
  // and the two nodes the edge lies between (a and b)
  auto interp = [&](int q, double& l, double& r, double& a, double& b) {
    const double* col = sP + q * NEXT + base;
    const double v0 = col[0], v1 = col[STEP], v2 = col[2 * STEP];
    const double v3 = col[3 * STEP], v4 = col[4 * STEP], v5 = col[5 * STEP];
    if constexpr (CENTRAL) {
      l = central4(v1, v2, v3, v4);
      r = l;
    } else {
      weno5_pair(v0, v1, v2, v3, v4, v5, eps4, l, r);
    }
    a = v2;
    b = v3;
  };
  // p and T first: their signs decide the first-order fallback, which is
  // then applied to each velocity component as soon as it is interpolated
  // (fewer values live at once).  The fallback takes the node values already
  // in registers (selects, no branch: a branch keeps both sets live)
  EdgeState<D> wl, wr;
  double lp, rp, lT, rT, pa, pb, Ta, Tb;
  interp(0, lp, rp, pa, pb);
  interp(1, lT, rT, Ta, Tb);
  const bool ok = (lp > 0.0) && (lT > 0.0) && (rp > 0.0) && (rT > 0.0);
  wl.p = ok ? lp : pa;
  wr.p = ok ? rp : pb;
  wl.T = ok ? lT : Ta;
  wr.T = ok ? rT : Tb;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double lu, ru, ua, ub;
    interp(2 + i, lu, ru, ua, ub);
    wl.u[i] = ok ? lu : ua;
    wr.u[i] = ok ? ru : ub;
  }
  // Rusanov flux (Eq. (11)-(12)), stored doubled, one variable at a time
  double rl, El, sl, rr, Er, sr;
  edge_thermo<D, J>(m, wl, rl, El, sl);
  edge_thermo<D, J>(m, wr, rr, Er, sr);
  const double S = fmax(sr, sl);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double UL, FL, UR, FR;
    edge_uf<D, J>(wl, rl, El, v, UL, FL);
    edge_uf<D, J>(wr, rr, Er, v, UR, FR);
    sF[v * NED + e] = fma(-S, UR - UL, FR + FL);
  }
}

// Physical flux of direction J (Eq. (1)-(3)) of one conserved edge state
// and its signal speed |u_J| + c (Eq. (7)), variable v of the flux in F[v].
template <int D, int J>
__device__ __forceinline__ void conserved_flux(const DevMesh& m, const double* U, double* F,
                                               double& speed) {
  const double ir = rcp_nr(U[0]);
  double u[D];
  double q2 = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    u[i] = U[1 + i] * ir;
    q2 = (i == 0) ? u[0] * u[0] : fma(u[i], u[i], q2);
  }
  const double p = m.gm1 * fma(-0.5 * U[0], q2, U[D + 1]);
  F[0] = U[1 + J];
#pragma unroll
  for (int i = 0; i < D; ++i) F[1 + i] = (i == J) ? fma(U[1 + i], u[J], p) : U[1 + i] * u[J];
  F[D + 1] = (U[D + 1] + p) * u[J];
  speed = sqrt_nr(m.gamma * p * ir) + fabs(u[J]);
}

// Riemann flux of direction J at one edge from characteristic variables (the
// shock-capturing variant of Section 2.2): the conserved states of the
// window nodes i-2 .. i+3 (in LDS, NEXT nodes per variable, STEP between
// neighbours along J) are projected on the left eigenvectors of the flux
// Jacobian A_J at the mean of nodes i and i+1, each characteristic field is
// interpolated by WENO5-JS (left value from i-2..i+2, right value from the
// mirrored stencil), and the edge states are projected back with the right
// eigenvectors.  Fields in the order u_J - c, entropy, shear (tangential
// directions ascending), u_J + c.  An edge where an interpolated rho or p is
// not positive on either side takes the states of nodes i and i+1.  The
// Rusanov flux (Eq. (11)-(12)) is stored doubled at sF[v NED + e].
template <int D, int J, int NEXT, int STEP, int NED>
__device__ __forceinline__ void edge_char(const DevMesh& m, const double* sP, int base, double* sF,
                                          int e) {
  constexpr int NV = D + 2;
  const double eps4 = 4.0 * m.eps;
  const double* col = sP + base;  // variable v of window node k at col[v NEXT + k STEP]
  // eigensystem at the mean state: u, c, 1/c, H = (E + p) / rho,
  // b1 = (gamma - 1) / c^2, b2 = b1 u.u / 2
  double ub[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    ub[v] = 0.5 * (col[v * NEXT + 2 * STEP] + col[v * NEXT + 3 * STEP]);
  const double ir = rcp_nr(ub[0]);
  double u[D];
  double q2 = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    u[i] = ub[1 + i] * ir;
    q2 = (i == 0) ? u[0] * u[0] : fma(u[i], u[i], q2);
  }
  const double pb = m.gm1 * fma(-0.5 * ub[0], q2, ub[D + 1]);
  double c, ic;
  sqrt_rsqrt_nr(m.gamma * pb * ir, c, ic);
  const double H = (ub[D + 1] + pb) * ir;
  const double b1 = m.gm1 * (ic * ic);
  const double b2 = 0.5 * b1 * q2;
  // per node, s = b1 (E - u.m) + b2 rho and a = (u_J rho - m_J) / c: the
  // acoustic fields are (s + a) / 2 (u_J - c) and (s - a) / 2 (u_J + c), the
  // entropy field rho - s; the shear field of a tangential t is m_t - u_t rho
  double sv[6], av[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double* nk = col + k * STEP;
    double um = u[0] * nk[NEXT];
#pragma unroll
    for (int i = 1; i < D; ++i) um = fma(u[i], nk[(1 + i) * NEXT], um);
    sv[k] = fma(b1, nk[(D + 1) * NEXT] - um, b2 * nk[0]);
    av[k] = fma(u[J], nk[0], -nk[(1 + J) * NEXT]) * ic;
  }
  double wl[NV], wr[NV];
  weno5_pair(0.5 * (sv[0] + av[0]), 0.5 * (sv[1] + av[1]), 0.5 * (sv[2] + av[2]),
             0.5 * (sv[3] + av[3]), 0.5 * (sv[4] + av[4]), 0.5 * (sv[5] + av[5]), eps4, wl[0],
             wr[0]);
  weno5_pair(0.5 * (sv[0] - av[0]), 0.5 * (sv[1] - av[1]), 0.5 * (sv[2] - av[2]),
             0.5 * (sv[3] - av[3]), 0.5 * (sv[4] - av[4]), 0.5 * (sv[5] - av[5]), eps4,
             wl[NV - 1], wr[NV - 1]);
  weno5_pair(col[0] - sv[0], col[STEP] - sv[1], col[2 * STEP] - sv[2], col[3 * STEP] - sv[3],
             col[4 * STEP] - sv[4], col[5 * STEP] - sv[5], eps4, wl[1], wr[1]);
  int f = 2;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    if (t == J) continue;
    const double* mt = col + (1 + t) * NEXT;
    weno5_pair(fma(-u[t], col[0], mt[0]), fma(-u[t], col[STEP], mt[STEP]),
               fma(-u[t], col[2 * STEP], mt[2 * STEP]), fma(-u[t], col[3 * STEP], mt[3 * STEP]),
               fma(-u[t], col[4 * STEP], mt[4 * STEP]), fma(-u[t], col[5 * STEP], mt[5 * STEP]),
               eps4, wl[f], wr[f]);
    ++f;
  }
  // back to conserved states: rho = W- + We + W+, m_J = u_J rho + c (W+ - W-),
  // m_t = u_t rho + W_t, E = H (W- + W+) + u_J c (W+ - W-) + q2/2 We + sum_t u_t W_t
  double UX[2][NV];
  bool ok = true;
#pragma unroll
  for (int X = 0; X < 2; ++X) {
    const double* w = X == 0 ? wl : wr;
    double* U = UX[X];
    const double A = w[0] + w[NV - 1];
    const double B = w[NV - 1] - w[0];
    const double rho = A + w[1];
    double Et = 0.5 * q2 * w[1];
    int g = 2;
#pragma unroll
    for (int t = 0; t < D; ++t) {
      if (t == J) {
        U[1 + t] = fma(u[J], rho, c * B);
      } else {
        U[1 + t] = fma(u[t], rho, w[g]);
        Et = fma(u[t], w[g], Et);
        ++g;
      }
    }
    U[0] = rho;
    U[D + 1] = fma(H, A, fma(u[J] * c, B, Et));
    const double irx = rcp_nr(rho);
    double ke = U[1] * (U[1] * irx);
#pragma unroll
    for (int i = 1; i < D; ++i) ke = fma(U[1 + i], U[1 + i] * irx, ke);
    const double px = m.gm1 * fma(-0.5, ke, U[D + 1]);
    ok = ok && (rho > 0.0) && (px > 0.0);
  }
  if (!ok) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      UX[0][v] = col[v * NEXT + 2 * STEP];
      UX[1][v] = col[v * NEXT + 3 * STEP];
    }
  }
  double FL[NV], FR[NV], sl, sr;
  conserved_flux<D, J>(m, UX[0], FL, sl);
  conserved_flux<D, J>(m, UX[1], FR, sr);
  const double S = fmax(sr, sl);
#pragma unroll
  for (int v = 0; v < NV; ++v) sF[v * NED + e] = fma(-S, UX[1][v] - UX[0][v], FR[v] + FL[v]);
}

// The scheme branch taken once per edge, so that each path is straight-line
// code the compiler can schedule across the primitives.  The characteristic
// scheme is a separate kernel instantiation (its LDS holds conserved states).
template <int D, int J, int NEXT, int STEP, int NED, bool CHAR>
__device__ __forceinline__ void edge_at(const DevMesh& m, const double* sP, int base, double* sF,
                                        int e) {
  if constexpr (CHAR)
    edge_char<D, J, NEXT, STEP, NED>(m, sP, base, sF, e);
  else if (m.scheme == AMR_SCHEME_CENTRAL)
    edge_at_scheme<D, J, NEXT, STEP, NED, true>(m, sP, base, sF, e);
  else
    edge_at_scheme<D, J, NEXT, STEP, NED, false>(m, sP, base, sF, e);
}


// Face fluxes G of direction J (flux form of Eq. (9)) from the edge fluxes
// in sF, their divergence into acc, and the patch-boundary faces into the
// flux registers.
template <int D, int TX, int TY, int TZ, int NT, int J>
__device__ __forceinline__ void cells_at(const double* sF, double* __restrict__ frp, int n,
                                         const int o[3], double acc[][D + 2], double inv_h,
                                         int wmask) {
  using S = TileShape<D, TX, TY, TZ>;
  constexpr int NV = D + 2;
  constexpr int G0 = S::T0 + (J == 0 ? 3 : 0);
  constexpr int G1 = S::T1 + (J == 1 ? 3 : 0);
  constexpr int G2 = S::T2 + (J == 2 ? 3 : 0);
  constexpr int NED = G0 * G1 * G2;
  constexpr int CPT = (S::NCELL + NT - 1) / NT;
  const int tid = threadIdx.x;
  const int nface = (D == 1) ? 1 : (D == 2 ? n : n * n);
  constexpr double c24 = 1.0 / 24.0;
  const double half_inv_h = 0.5 * inv_h;
  // patch-boundary faces whose flux registers refluxing reads
  const bool lo_reg = (wmask >> (2 * J)) & 1, hi_reg = (wmask >> (2 * J + 1)) & 1;
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc) {
    const int cell = tid + cc * NT;
    if (cell >= S::NCELL) break;
    const int t0 = cell % S::T0;
    const int t1 = (cell / S::T0) % S::T1;
    const int t2 = cell / (S::T0 * S::T1);
    const int tj = J == 0 ? t0 : (J == 1 ? t1 : t2);
    // edge-array index of edge (t_J - 2 + k) + 1/2 in the edge box
    int eb;
    constexpr int ESTEP = J == 0 ? 1 : (J == 1 ? G0 : G0 * G1);
    if constexpr (J == 0) eb = G0 * (t1 + G1 * t2);
    else if constexpr (J == 1) eb = t0 + G0 * G1 * t2;
    else eb = t0 + G0 * t1;
    eb += tj * ESTEP;
    const int i = o[J] + tj;
    int tang = 0;
    if constexpr (D == 2) tang = (J == 0) ? (o[1] + t1) : (o[0] + t0);
    if constexpr (D == 3) {
      if constexpr (J == 0) tang = (o[1] + t1) + __mul24(n, o[2] + t2);
      else if constexpr (J == 1) tang = (o[0] + t0) + __mul24(n, o[2] + t2);
      else tang = (o[0] + t0) + __mul24(n, o[1] + t1);
    }
    // the flux registers of this face (variable v at v nface + tang of the
    // face's block; 32-bit offsets, 24-bit products), written per variable
    const bool lo = i == 0 && lo_reg, hi = i == n - 1 && hi_reg;
    double* fb = frp + __mul24((J * 2 + (hi ? 1 : 0)) * NV, nface) + tang;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      // edge fluxes are stored doubled (the Rusanov 1/2 is applied here, as
      // 1/2 inv_h, and to the boundary faces; power-of-two scaling is exact)
      const double* F = sF + v * NED + eb;
      const double Fm2 = F[0], Fm1 = F[ESTEP], F0 = F[2 * ESTEP], Fp1 = F[3 * ESTEP];
      const double Gp = fma(-c24, fma(-2.0, F0, Fm1) + Fp1, F0);
      const double Gm = fma(-c24, fma(-2.0, Fm1, Fm2) + F0, Fm1);
      acc[cc][v] = fma(-(Gp - Gm), half_inv_h, acc[cc][v]);
      if (lo || hi) fb[__mul24(v, nface)] = 0.5 * (hi ? Gp : Gm);
    }
  }
}

// Riemann flux at every edge i+1/2, i = o_J-2 .. o_J+T_J, of direction J
// from the node values in sP (the union layout in 1D/2D, the tile extended
// along J in 3D), into sF.
template <int D, int TX, int TY, int TZ, int NT, int J, bool UNION, bool CHAR>
__device__ __forceinline__ void edges_dir(const DevMesh& m, const double* sP, double* sF) {
  using S = TileShape<D, TX, TY, TZ>;
  // E0 is the row pitch of the node array
  constexpr int E0 = UNION ? S::UPITCH : S::xpitch(J);
  constexpr int E1 = UNION ? (D >= 2 ? S::T1 + 8 : 1) : S::T1 + (J == 1 ? 8 : 0);
  constexpr int E2 = UNION ? 1 : S::T2 + (J == 2 ? 8 : 0);
  constexpr int NEXT = E0 * E1 * E2;
  constexpr int G0 = S::T0 + (J == 0 ? 3 : 0);
  constexpr int G1 = S::T1 + (J == 1 ? 3 : 0);
  constexpr int G2 = S::T2 + (J == 2 ? 3 : 0);
  constexpr int NED = G0 * G1 * G2;
  constexpr int STEP = J == 0 ? 1 : (J == 1 ? E0 : E0 * E1);
  for (int t = threadIdx.x; t < NED; t += NT) {
    // 3D x edges go to the lanes cross-section first: the 16 lanes of an LDS
    // pass then read rows r..r+15 of the odd-pitched node box and write
    // edges a0 + 11 r (distinct banks); row by row, 11 edges to a row, they
    // would collide
    constexpr bool XCROSS = !UNION && J == 0;
    const int a0 = XCROSS ? t / (G1 * G2) : t % G0;
    const int a1 = XCROSS ? t % G1 : (t / G0) % G1;
    const int a2 = XCROSS ? (t / G1) % G2 : t / (G0 * G1);
    const int e = XCROSS ? a0 + G0 * (a1 + G1 * a2) : t;
    // layout index of node i-2 of this edge's window
    int base;
    if constexpr (!UNION) base = a0 + E0 * (a1 + E1 * a2);
    else if constexpr (J == 0) base = (D >= 2 ? (a1 + 4) * E0 : 0) + a0;
    else base = a1 * E0 + (a0 + 4);
    edge_at<D, J, NEXT, STEP, NED, CHAR>(m, sP, base, sF, e);
  }
}

// 3D, characteristic scheme: the conserved values of the tile extended by 4
// nodes on both sides along J, into sP in the extended-box layout.  The
// tile's own nodes come first in the thread order and the 8 halo layers
// after them, so that a wave holds nodes of one kind (the tile's own nodes
// are read straight from the patch); every thread issues the loads of all
// its nodes before storing any.
template <int D, int TX, int TY, int TZ, int NT, int J, bool FUSE>
__device__ __forceinline__ void load_dir(const DevMesh& m, const double* __restrict__ Uin,
                                         const double* __restrict__ Pin, int n, int full,
                                         const int o[3], const int pc[3], int l,
                                         const long long* sN, double* sP) {
  using S = TileShape<D, TX, TY, TZ>;
  constexpr int NV = D + 2;
  constexpr int E0 = S::xpitch(J);             // row pitch
  constexpr int E1 = S::T1 + (J == 1 ? 8 : 0);
  constexpr int E2 = S::T2 + (J == 2 ? 8 : 0);
  constexpr int NEXT = E0 * E1 * E2;
  constexpr int NC = S::NCELL;
  constexpr int TJ = J == 0 ? S::T0 : (J == 1 ? S::T1 : S::T2);
  constexpr int HL = NC / TJ;                  // nodes of one layer across J
  constexpr int CA = J == 0 ? S::T1 : S::T0;   // extent of the lower cross direction
  constexpr int NNODE = NC + 8 * HL;           // nodes of the extended box
  constexpr int ITER = (NNODE + NT - 1) / NT;
  double u[ITER][NV];
  int lidx[ITER];
#pragma unroll
  for (int k = 0; k < ITER; ++k) {
    const int idx = threadIdx.x + k * NT;
    lidx[k] = -1;
    if (idx >= NNODE) continue;
    int t[3];
    if (idx < NC) {
      t[0] = idx % S::T0;
      t[1] = (idx / S::T0) % S::T1;
      t[2] = idx / (S::T0 * S::T1);
    } else {
      const int hh = idx - NC;
      const int layer = hh / HL;                // -4..-1, then T_J..T_J+3
      const int r = hh - layer * HL;
      const int a = r % CA, b = r / CA;         // the two other directions, lower first
      t[J] = layer < 4 ? layer - 4 : TJ + layer - 4;
      t[J == 0 ? 1 : 0] = a;
      t[J == 2 ? 1 : 2] = b;
    }
    const int c[3] = {o[0] + t[0], o[1] + t[1], o[2] + t[2]};
    lidx[k] = (t[0] + (J == 0 ? 4 : 0)) + E0 * ((t[1] + (J == 1 ? 4 : 0)) +
                                                E1 * (t[2] + (J == 2 ? 4 : 0)));
    node_conserved_dir<D, J, FUSE>(m, Uin, Pin, n, full, c, pc, l, sN, u[k]);
  }
#pragma unroll
  for (int k = 0; k < ITER; ++k)
    if (lidx[k] >= 0) node_store<D, true>(m, u[k], sP, NEXT, lidx[k]);
}

// 3D primitive schemes: thread t < NCELL loads the conserved values of tile
// node t once, first in the item (they need no neighbour table), and keeps
// them in `keep` for the three directions and as the stage input of cell t
// in the epilogue.
template <int D, int TX, int TY, int TZ>
__device__ __forceinline__ void own_load(const double* __restrict__ Pin, int full, const int o[3],
                                         double* keep) {
  using S = TileShape<D, TX, TY, TZ>;
  const int tid = threadIdx.x;
  if (tid < S::NCELL) {
    const int t0 = tid % S::T0, t1 = (tid / S::T0) % S::T1, t2 = tid / (S::T0 * S::T1);
    const int off = box_off<D>(full, o[0] + t0 + NG, o[1] + t1 + NG, o[2] + t2 + NG);
    const int vs = var_stride<D>(full);
#pragma unroll
    for (int v = 0; v < D + 2; ++v) keep[v] = Pin[v * vs + off];
  }
}

// 3D primitive schemes: the 8 halo layers of the tile extended along J (its
// own nodes are kept in registers).  For y and z their loads are issued
// (halo_issue) before the previous direction's divergence is formed and
// converted and stored (halo_store) after it, so that they are in flight
// meanwhile.  Halo node h (layers -4..-1, then T_J..T_J+3, the two other
// directions lower first) is item h / NT of thread h mod NT.
template <int D, int TX, int TY, int TZ, int NT, int J>
struct DirHalo {
  using S = TileShape<D, TX, TY, TZ>;
  static constexpr int NV = D + 2;
  static constexpr int TJ = J == 0 ? S::T0 : (J == 1 ? S::T1 : S::T2);
  static constexpr int HL = S::NCELL / TJ;                  // nodes of one layer
  static constexpr int NH = 8 * HL;
  static constexpr int ITER = (NH + NT - 1) / NT;
  double u[ITER][NV];
  int lidx[ITER];
};

template <int D, int TX, int TY, int TZ, int NT, int J, bool FUSE>
__device__ __forceinline__ void halo_issue(const DevMesh& m, const double* __restrict__ Uin,
                                           const double* __restrict__ Pin, int n, int full,
                                           const int o[3], const int pc[3], int l,
                                           const long long* sN,
                                           DirHalo<D, TX, TY, TZ, NT, J>& h) {
  using S = TileShape<D, TX, TY, TZ>;
  using H = DirHalo<D, TX, TY, TZ, NT, J>;
  constexpr int E0 = S::xpitch(J);
  constexpr int E1 = S::T1 + (J == 1 ? 8 : 0);
  constexpr int CA = J == 0 ? S::T1 : S::T0;   // extent of the lower cross direction
  const int tid = phase_tid();
#pragma unroll
  for (int k = 0; k < H::ITER; ++k) {
    // threads past the last halo node load node NH - 1 again (no branch
    // around the loads) and store nothing
    const int h0 = tid + k * NT;
    const int hh = h0 < H::NH ? h0 : H::NH - 1;
    const int layer = hh / H::HL;
    const int r = hh - layer * H::HL;
    int t[3];
    t[J] = layer < 4 ? layer - 4 : H::TJ + layer - 4;
    t[J == 0 ? 1 : 0] = r % CA;
    t[J == 2 ? 1 : 2] = r / CA;
    const int c[3] = {o[0] + t[0], o[1] + t[1], o[2] + t[2]};
    h.lidx[k] = h0 < H::NH ? (t[0] + (J == 0 ? 4 : 0)) +
                                 E0 * ((t[1] + (J == 1 ? 4 : 0)) + E1 * (t[2] + (J == 2 ? 4 : 0)))
                           : -1;
    node_conserved_dir<D, J, FUSE>(m, Uin, Pin, n, full, c, pc, l, sN, h.u[k]);
  }
}

template <int D, int TX, int TY, int TZ, int NT, int J>
__device__ __forceinline__ void halo_store(const DevMesh& m, const DirHalo<D, TX, TY, TZ, NT, J>& h,
                                           const double* keep, double* sP) {
  using S = TileShape<D, TX, TY, TZ>;
  using H = DirHalo<D, TX, TY, TZ, NT, J>;
  constexpr int E0 = S::xpitch(J);
  constexpr int E1 = S::T1 + (J == 1 ? 8 : 0);
  constexpr int NEXT = S::ext(J);
  const int tid = phase_tid();
  if (tid < S::NCELL) {
    const int t0 = tid % S::T0, t1 = (tid / S::T0) % S::T1, t2 = tid / (S::T0 * S::T1);
    node_store<D, false>(m, keep, sP, NEXT,
                         (t0 + (J == 0 ? 4 : 0)) +
                             E0 * ((t1 + (J == 1 ? 4 : 0)) + E1 * (t2 + (J == 2 ? 4 : 0))));
  }
#pragma unroll
  for (int k = 0; k < H::ITER; ++k)
    if (h.lidx[k] >= 0) node_store<D, false>(m, h.u[k], sP, NEXT, h.lidx[k]);
}

// 1D/2D: edge fluxes and their divergence for direction J from the union
// layout loaded once for all directions.
template <int D, int TX, int TY, int TZ, int NT, int J, bool CHAR>
__device__ __forceinline__ void stage_direction(const DevMesh& m, double* __restrict__ frp, int n,
                                                const int o[3], double* sP, double* sF,
                                                double acc[][D + 2], double inv_h, int wmask) {
  edges_dir<D, TX, TY, TZ, NT, J, true, CHAR>(m, sP, sF);
  __syncthreads();
  cells_at<D, TX, TY, TZ, NT, J>(sF, frp, n, o, acc, inv_h, wmask);
  __syncthreads();
}

// 2D union layout, both directions at once: the x and y edges form one work
// range (x first), then every cell takes its x and then its y divergence,
// the order of the direction-by-direction path.
template <int D, int TX, int TY, int NT, bool CHAR>
__device__ __forceinline__ void stage_both(const DevMesh& m, double* __restrict__ frp, int n,
                                           const int o[3], const double* sP, double* sFx,
                                           double* sFy, double acc[][D + 2], double inv_h,
                                           int wmask) {
  static_assert(D == 2, "combined sweep is 2D");
  using S = TileShape<D, TX, TY, 1>;
  constexpr int E0 = S::UPITCH;                // row pitch of the union box
  constexpr int NEXT = S::NUNION;
  constexpr int GX0 = S::T0 + 3, NEDX = GX0 * S::T1;
  constexpr int GY0 = S::T0, NEDY = S::T0 * (S::T1 + 3);
  for (int e = threadIdx.x; e < NEDX + NEDY; e += NT) {
    if (e < NEDX) {
      const int a0 = e % GX0, a1 = e / GX0;
      edge_at<D, 0, NEXT, 1, NEDX, CHAR>(m, sP, (a1 + 4) * E0 + a0, sFx, e);
    } else {
      const int f = e - NEDX;
      const int a0 = f % GY0, a1 = f / GY0;
      edge_at<D, 1, NEXT, E0, NEDY, CHAR>(m, sP, a1 * E0 + (a0 + 4), sFy, f);
    }
  }
  __syncthreads();
  cells_at<D, TX, TY, 1, NT, 0>(sFx, frp, n, o, acc, inv_h, wmask);
  cells_at<D, TX, TY, 1, NT, 1>(sFy, frp, n, o, acc, inv_h, wmask);
}

// One (pid, tile) work item: the whole RHS of the tile and its stage
// combination; `best` collects the CFL rate bits of the item's cells.
// Restriction of a finest-level tile into its parent patch, from the new
// values of its cells (sR: variable v of tile cell i at sR[v NCELL + i]):
// each parent cell is the mean of its 2^D children, summed as the
// post-stage restriction sums them (x pairs first, then y, then z).  The
// finest level is never the coarse side of a coarse/fine face, so its values
// are final once the stage kernel has written them.  SERIAL: one variable
// at a time (unrolled, the reads of all variables are issued at once and can
// take more registers than the primitive schemes' kernels have).
template <int D, int TX, int TY, int TZ, int NT, bool SERIAL>
__device__ __forceinline__ void restrict_tile(const DevMesh& m, double* __restrict__ out, int pid,
                                              int l, const int o[3], const double* sR) {
  using S = TileShape<D, TX, TY, TZ>;
  constexpr int NV = D + 2;
  constexpr int NC = S::NCELL;
  constexpr int H0 = S::T0 / 2, H1 = D >= 2 ? S::T1 / 2 : 1, H2 = D >= 3 ? S::T2 / 2 : 1;
  constexpr int NP = H0 * H1 * H2;
  static_assert(S::T0 % 2 == 0 && (D < 2 || S::T1 % 2 == 0) && (D < 3 || S::T2 % 2 == 0),
                "tiles cover whole 2^D groups of children");
  const int ppid = m.parent[pid];
  const LevelC& C = m.lv[l - 1];
  const int h = m.lv[l].n / 2;
  double* Pp = out + patch_base(m, ppid, l - 1);
  const int vsc = var_stride<D>(C.full);
  for (int k = threadIdx.x; k < NP; k += NT) {
    const int a = k % H0, b = (k / H0) % H1, c = k / (H0 * H1);
    int q[3] = {0, 0, 0};
#pragma unroll
    for (int j = 0; j < D; ++j)
      q[j] = m.coord[3 * pid + j] * h - m.coord[3 * ppid + j] * C.n + o[j] / 2 + (j == 0 ? a : (j == 1 ? b : c)) + NG;
    const int dst = box_off<D>(C.full, q[0], q[1], q[2]);
    auto at = [&](int v, int x, int y, int z) {
      return sR[v * NC + (2 * a + x) + S::T0 * ((2 * b + y) + S::T1 * (2 * c + z))];
    };
    auto one = [&](int v) {
      auto xsum = [&](int y, int z) { return at(v, 0, y, z) + at(v, 1, y, z); };
      double r;
      if constexpr (D == 1) r = xsum(0, 0) * 0.5;
      else if constexpr (D == 2) r = (xsum(0, 0) + xsum(1, 0)) * 0.25;
      else r = ((xsum(0, 0) + xsum(1, 0)) + (xsum(0, 1) + xsum(1, 1))) * 0.125;
      Pp[v * vsc + dst] = r;
    };
    if constexpr (SERIAL) {
#pragma unroll 1
      for (int v = 0; v < NV; ++v) one(v);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) one(v);
    }
  }
}

template <int D, int TX, int TY, int TZ, int NT, bool FUSE, bool BOTH, bool CHAR>
__device__ __forceinline__ void stage_item(const DevMesh& m, int mode,
                                           const double* __restrict__ Uin, const double* Un,
                                           double* out, double* __restrict__ fr,
                                           const int* __restrict__ tiles, int item,
                                           const double* __restrict__ dtp,
                                           unsigned long long* __restrict__ lam_next,
                                           const uint8_t* __restrict__ cfmask,
                                           const unsigned long long* __restrict__ lam_in,
                                           double* __restrict__ dt_out, double* sP, double* sF,
                                           long long* sN, unsigned long long& best) {
  using S = TileShape<D, TX, TY, TZ>;
  constexpr int NV = D + 2;
  constexpr int CPT = (S::NCELL + NT - 1) / NT;
  constexpr bool UNION = D <= 2;
  const int pid = tiles[2 * item];
  const int tix = tiles[2 * item + 1];
  const int l = m.level[pid];
  const LevelC& L = m.lv[l];
  const int n = L.n, full = L.full;
  const int nt0 = n / S::T0, nt1 = n / S::T1;
  const int o[3] = {(tix % nt0) * S::T0, ((tix / nt0) % nt1) * S::T1, (tix / (nt0 * nt1)) * S::T2};
  const long long base = patch_base(m, pid, l);
  const double* Pin = Uin + base;
  double* frp = fr + L.fr_off + (long long)(pid - L.pid_base) * L.fr_stride;
  // faces whose flux registers are written (the second half of the mask array)
  const int wmask = cfmask[m.max_patches + pid];
  double acc[CPT][NV];
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[cc][v] = 0.0;

  const int pc[3] = {m.coord[3 * pid], m.coord[3 * pid + 1], m.coord[3 * pid + 2]};
  // 3D primitive schemes: the conserved values of this thread's tile node,
  // loaded first (their loads need no neighbour table) and kept for the three
  // directions and the epilogue (own_load), and U^n of its cell
  constexpr bool KEPT = !UNION && !CHAR;
  double keep[NV], un0[NV];
  static_assert(!KEPT || NT >= S::NCELL, "a thread per tile node holds its values");
  if constexpr (KEPT) own_load<D, TX, TY, TZ>(Pin, full, o, keep);
  if constexpr (FUSE) {
    load_neighbours<D>(m, l, pc, sN);
    __syncthreads();
  }
  if constexpr (UNION) {
    load_union<D, TX, TY, NT, FUSE, CHAR>(m, Uin, Pin, n, full, o, pc, l, sN, sP);
    __syncthreads();
    if constexpr (BOTH && D == 2) {
      stage_both<D, TX, TY, NT, CHAR>(m, frp, n, o, sP, sF,
                                      sF + (D + 2) * ((S::T0 + 3) * S::T1), acc, L.inv_h, wmask);
    } else {
      stage_direction<D, TX, TY, TZ, NT, 0, CHAR>(m, frp, n, o, sP, sF, acc, L.inv_h, wmask);
      if constexpr (D >= 2)
        stage_direction<D, TX, TY, TZ, NT, 1, CHAR>(m, frp, n, o, sP, sF, acc, L.inv_h, wmask);
    }
  } else {
    // 3D, direction by direction: the next direction's nodes are loaded in
    // the phase that forms the previous direction's divergence (sP is free
    // once the edges are done, sF is read), two block barriers per direction
    if constexpr (KEPT) {
      DirHalo<D, TX, TY, TZ, NT, 0> h;
      halo_issue<D, TX, TY, TZ, NT, 0, FUSE>(m, Uin, Pin, n, full, o, pc, l, sN, h);
      halo_store<D, TX, TY, TZ, NT, 0>(m, h, keep, sP);
    } else {
      load_dir<D, TX, TY, TZ, NT, 0, FUSE>(m, Uin, Pin, n, full, o, pc, l, sN, sP);
    }
    __syncthreads();
    edges_dir<D, TX, TY, TZ, NT, 0, false, CHAR>(m, sP, sF);
    __syncthreads();
    if constexpr (KEPT) {
      DirHalo<D, TX, TY, TZ, NT, 1> h;
      halo_issue<D, TX, TY, TZ, NT, 1, FUSE>(m, Uin, Pin, n, full, o, pc, l, sN, h);
      cells_at<D, TX, TY, TZ, NT, 0>(sF, frp, n, o, acc, L.inv_h, wmask);
      halo_store<D, TX, TY, TZ, NT, 1>(m, h, keep, sP);
    } else {
      load_dir<D, TX, TY, TZ, NT, 1, FUSE>(m, Uin, Pin, n, full, o, pc, l, sN, sP);
      cells_at<D, TX, TY, TZ, NT, 0>(sF, frp, n, o, acc, L.inv_h, wmask);
    }
    __syncthreads();
    edges_dir<D, TX, TY, TZ, NT, 1, false, CHAR>(m, sP, sF);
    __syncthreads();
    if constexpr (KEPT) {
      DirHalo<D, TX, TY, TZ, NT, 2> h;
      halo_issue<D, TX, TY, TZ, NT, 2, FUSE>(m, Uin, Pin, n, full, o, pc, l, sN, h);
      cells_at<D, TX, TY, TZ, NT, 1>(sF, frp, n, o, acc, L.inv_h, wmask);
      halo_store<D, TX, TY, TZ, NT, 2>(m, h, keep, sP);
    } else {
      load_dir<D, TX, TY, TZ, NT, 2, FUSE>(m, Uin, Pin, n, full, o, pc, l, sN, sP);
      cells_at<D, TX, TY, TZ, NT, 1>(sF, frp, n, o, acc, L.inv_h, wmask);
    }
    __syncthreads();
    edges_dir<D, TX, TY, TZ, NT, 2, false, CHAR>(m, sP, sF);
    __syncthreads();
    if constexpr (KEPT) {
      // U^n of the thread's own cell for the combination, loaded while the
      // last divergence is formed (the kept stage input when U^n is it)
      const int tid = threadIdx.x;
      if (mode != kModeRHS && tid < S::NCELL) {
        if (Un == Uin) {
#pragma unroll
          for (int v = 0; v < NV; ++v) un0[v] = keep[v];
        } else {
          const int t0 = tid % S::T0, t1 = (tid / S::T0) % S::T1, t2 = tid / (S::T0 * S::T1);
          const double* p = Un + base + box_off<D>(full, o[0] + t0 + NG, o[1] + t1 + NG,
                                                   o[2] + t2 + NG);
          const int vs = var_stride<D>(full);
#pragma unroll
          for (int v = 0; v < NV; ++v) un0[v] = __builtin_nontemporal_load(p + v * vs);
        }
      }
    }
    cells_at<D, TX, TY, TZ, NT, 2>(sF, frp, n, o, acc, L.inv_h, wmask);
  }

  const int vs = var_stride<D>(full);
  // stage 1 of a step may take dt = CFL / rate from the rate slot itself
  // (every block computes it; the first work item publishes it for the rest
  // of the step and clears the slot stage 3 accumulates into)
  double dt;
  if (mode == kModeRHS) {
    dt = 0.0;
  } else if (lam_in) {
    dt = m.cfl / __longlong_as_double((long long)lam_in[0]);
    if (item == 0 && threadIdx.x == 0) {
      dt_out[0] = dt;
      lam_next[0] = 0ull;
    }
  } else {
    dt = dtp[0];
  }
  constexpr double c23 = 2.0 / 3.0;
  // next step's CFL rate from the final leaf values; cells on coarse/fine
  // faces are left to the flux-correction kernel, which changes them
  const bool want_rate = lam_next != nullptr && mode == kModeStage3;
  const int fmask = want_rate ? cfmask[pid] : 0;
  // a tile of the finest level is restricted into its parent here, from the
  // values it writes (staged in sF, free once every thread has read its
  // edge fluxes)
  const bool restrict_here = mode != kModeRHS && l == m.nlev - 1 && l >= 1;
  static_assert(S::NCELL <= S::EDMAX, "the staged cell values fit sF");
  double* sR = sF;
  if (restrict_here) __syncthreads();
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc) {
    const int cell = threadIdx.x + cc * NT;
    if (cell >= S::NCELL) break;
    const int t0 = cell % S::T0;
    const int t1 = (cell / S::T0) % S::T1;
    const int t2 = cell / (S::T0 * S::T1);
    const long long off = base + box_off<D>(full, o[0] + t0 + NG, o[1] + t1 + NG, o[2] + t2 + NG);
    double r[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const long long a = off + v * vs;
      const double Lv = acc[cc][v];
      if (mode == kModeRHS) {
        r[v] = Lv;
      } else if (mode == kModeStage1) {
        // U^n and the stage input of the cell: held for the thread's own
        // cell (cc = 0) in 3D, else loaded
        const double un = (KEPT && cc == 0) ? un0[v] : Un[a];
        r[v] = fma(dt, Lv, un);
      } else {
        const double un = (KEPT && cc == 0) ? un0[v] : Un[a];
        const double ui = (KEPT && cc == 0) ? keep[v] : Uin[a];
        r[v] = fma(mode == kModeStage2 ? 0.25 : c23, fma(dt, Lv, ui) - un, un);
      }
      // 3D: a non-temporal store, which keeps the stage input's halo rows
      // in L2 for the neighbouring tiles
      if constexpr (UNION)
        out[a] = r[v];
      else
        __builtin_nontemporal_store(r[v], out + a);
      if (restrict_here) sR[v * S::NCELL + cell] = r[v];
    }
    if (want_rate) {
      const int c3[3] = {o[0] + t0, o[1] + t1, o[2] + t2};
      bool on_cf = false;
      for (int j = 0; j < D; ++j)
        on_cf |= ((fmask >> (2 * j)) & 1) && c3[j] == 0 || ((fmask >> (2 * j + 1)) & 1) && c3[j] == n - 1;
      if (!on_cf) {
        const unsigned long long bits = cell_rate_bits<D>(r, m, L.h);
        best = bits > best ? bits : best;
      }
    }
  }
  if (restrict_here) {
    __syncthreads();
    restrict_tile<D, TX, TY, TZ, NT, KEPT>(m, out, pid, l, o, sR);
  }
}

// The fused stage kernel over (pid, tile) work items, one item per block.
// With `dir` (batched launches) the list and its live count are read from
// the device list directory {offset into `tiles`, count}, so that a launch
// recorded once stays valid when a regrid rewrites the lists (its grid may
// then hold more blocks than items).  XCD x (block b runs on XCD b mod 8)
// takes one contiguous eighth of the list, which is in brick order, so the
// items in flight on an XCD are neighbours that read each other's cells as
// halos from that XCD's L2.
template <int D, int TX, int TY, int TZ, int NT, bool FUSE, bool BOTH, bool CHAR>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(CHAR ? 4 : 6))) void k_stage(DevMesh m, int mode, const double* __restrict__ Uin,
                                              const double* Un, double* out,
                                              double* __restrict__ fr,
                                              const int* __restrict__ tiles, int count,
                                              const int* __restrict__ dir,
                                              const double* __restrict__ dtp,
                                              unsigned long long* __restrict__ lam_next,
                                              const uint8_t* __restrict__ cfmask,
                                              const unsigned long long* __restrict__ lam_in,
                                              double* __restrict__ dt_out) {
  using S = TileShape<D, TX, TY, TZ>;
  constexpr bool UNION = D <= 2;
  constexpr int NU = S::NUNION;
  // edge fluxes: one direction at a time, or x and y together (BOTH)
  constexpr int NEDXY = (S::T0 + 3) * S::T1 + S::T0 * (S::T1 + 3);
  __shared__ double sP[(D + 2) * (UNION ? NU : S::EXTMAX)];
  __shared__ double sF[(D + 2) * (BOTH ? NEDXY : S::EDMAX)];
  __shared__ long long sN[27];
  const int* list = dir ? tiles + dir[0] : tiles;
  const int item = xcd_item(dir ? dir[1] : count);
  if (item < 0) return;
  unsigned long long best = 0ull;
  stage_item<D, TX, TY, TZ, NT, FUSE, BOTH, CHAR>(m, mode, Uin, Un, out, fr, list, item, dtp,
                                                  lam_next, cfmask, lam_in, dt_out, sP, sF, sN,
                                                  best);
  if (lam_next != nullptr && mode == kModeStage3) block_max_atomic(best, lam_next);
}

}  // namespace

// Tile variants: thread counts cover the edges of one direction of the
// tile in one pass (multiples of 64); the 8x8x8 tile's 704 edges take 768
// threads, 12 waves, which spread evenly over a CU's 4 SIMDs (with 11 waves
// one SIMD holds a wave less of every block: 13.1 against 14.6 ms per RHS
// launch over 156 M cells of a four-level 3D hierarchy).
static const Kernels::TileVariant kVariants[] = {
    {1, 16, 1, 1, 64}, {1, 8, 1, 1, 64},                                   // 1D
    {2, 16, 16, 1, 320}, {2, 16, 8, 1, 192}, {2, 8, 8, 1, 128},           // 2D
    {3, 8, 8, 8, 768}, {3, 8, 8, 4, 448}, {3, 4, 4, 4, 128},              // 3D
    // 2D, x and y edges in one sweep (stage_both)
    {2, 16, 16, 1, 320, 1}, {2, 16, 8, 1, 192, 1}, {2, 8, 8, 1, 128, 1},
};

int Kernels::num_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

Kernels::TileVariant Kernels::variant(int v) { return kVariants[v]; }

bool Kernels::variant_fits(int v, int dim, const int* n, int nlev) {
  if (v < 0 || v >= num_variants() || kVariants[v].dim != dim) return false;
  const TileVariant& t = kVariants[v];
  for (int l = 0; l < nlev; ++l) {
    if (n[l] % t.tx) return false;
    if (dim >= 2 && n[l] % t.ty) return false;
    if (dim >= 3 && n[l] % t.tz) return false;
  }
  return true;
}

int Kernels::default_variant(int dim, const int* n, int nlev) {
  for (int v = 0; v < num_variants(); ++v)
    if (variant_fits(v, dim, n, nlev)) return v;
  return -1;
}

int Kernels::tiles_per_patch(int v, int n) {
  const TileVariant& t = kVariants[v];
  int r = n / t.tx;
  if (t.dim >= 2) r *= n / t.ty;
  if (t.dim >= 3) r *= n / t.tz;
  return r;
}

void Kernels::stage(const DevMesh& m, int mode, const double* Uin, const double* Un,
                    double* out, double* fr, const int* tiles, int count, const int* dir,
                    const double* dt, bool fuse, unsigned long long* lam_next,
                    const uint8_t* cfmask, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                    const unsigned long long* lam_in, double* dt_out) {
  if (count <= 0) return;
  // one block per work item (`count` may exceed the live count read from the
  // directory), in whole groups of kXcds blocks (see xcd_item)
  const int nb = stage_grid(count);
  const bool chr = m.scheme == AMR_SCHEME_CHAR;
#define AMR_STAGE_K(D, TX, TY, TZ, NT, F, B, C)                                                \
  do {                                                                                          \
    auto kern = k_stage<D, TX, TY, TZ, NT, F, B, C>;                                            \
    if (ev0)                                                                                    \
      hipExtLaunchKernelGGL(kern, dim3(nb), dim3(NT), 0, s, ev0, ev1, 0, m, mode, Uin, Un,  \
                            out, fr, tiles, count, dir, dt, lam_next, cfmask, lam_in, dt_out);  \
    else                                                                                        \
      hipLaunchKernelGGL(kern, dim3(nb), dim3(NT), 0, s, m, mode, Uin, Un, out, fr, tiles, \
                         count, dir, dt, lam_next, cfmask, lam_in, dt_out);                     \
  } while (0)
#define AMR_STAGE_F(D, TX, TY, TZ, NT, F, B)          \
  do {                                                \
    if (chr)                                          \
      AMR_STAGE_K(D, TX, TY, TZ, NT, F, B, true);     \
    else                                              \
      AMR_STAGE_K(D, TX, TY, TZ, NT, F, B, false);    \
  } while (0)
#define AMR_STAGE(D, TX, TY, TZ, NT, B)        \
  do {                                         \
    if (fuse)                                  \
      AMR_STAGE_F(D, TX, TY, TZ, NT, true, B); \
    else                                       \
      AMR_STAGE_F(D, TX, TY, TZ, NT, false, B);\
  } while (0)
  switch (m.tile) {
    case 0: AMR_STAGE(1, 16, 1, 1, 64, false); break;
    case 1: AMR_STAGE(1, 8, 1, 1, 64, false); break;
    case 2: AMR_STAGE(2, 16, 16, 1, 320, false); break;
    case 3: AMR_STAGE(2, 16, 8, 1, 192, false); break;
    case 4: AMR_STAGE(2, 8, 8, 1, 128, false); break;
    case 5: AMR_STAGE(3, 8, 8, 8, 768, false); break;
    case 6: AMR_STAGE(3, 8, 8, 4, 448, false); break;
    case 7: AMR_STAGE(3, 4, 4, 4, 128, false); break;
    case 8: AMR_STAGE(2, 16, 16, 1, 320, true); break;
    case 9: AMR_STAGE(2, 16, 8, 1, 192, true); break;
    default: AMR_STAGE(2, 8, 8, 1, 128, true); break;
  }
#undef AMR_STAGE
#undef AMR_STAGE_F
#undef AMR_STAGE_K
}

}  // namespace amr
