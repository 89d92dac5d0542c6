// Slope limiter for basis orders >= 1 (Sec. 2.3 names the minmod limiter of van Leer
// 1979 and the scaling limiter of Moe, Rossmanith & Seal 2015 for the p >= 1 shock
// runs): minmod-bounded slopes applied as one scaling factor per element.
//
// The stage launch ahead of it (k_element in MODE_STAGE_LIM) writes the unlimited
// stage, its element averages ([var][element]) and its primitives.
// k_limit   per element: for each component k and direction d the slope s, the
//           coefficient of xi_d in the element's Legendre expansion (sum_n w_n
//           xi_{d,n} u_n / sum_n w_n xi_{d,n}^2, mirror nodes paired so that a constant
//           element has slope exactly 0), and its bound s~ = minmod(s, ubar_+ - ubar,
//           ubar - ubar_-) by the neighbours' averages (periodic wrap, the element's
//           own average at a non-periodic end); theta = the least s~ / s over the pairs
//           where |s - s~| exceeds kLimEps times the component's scale (the average
//           energy E = |tau + D c^2| over c^2 for D, over c for S, E for tau); where
//           theta < 1 every node moves to ubar + theta (u - ubar).  Then the
//           physicality operator (Sec. 2.5); U and the next stage's primitives are
//           written only for the nodes that changed (the stage launch wrote both for
//           every node).  One factor for all components keeps every node on the
//           segment to the (admissible) average.
//
// Workgroup layout: four waves, each holding EPW = 64 / NPE whole elements (one node
// per lane, the lanes past EPW * NPE idle), so that every exchange among an element's
// nodes stays inside one wave and needs no workgroup barrier; each lane has its own
// LDS slot (its thread index).  The (direction, component) pairs of an element are
// spread over its lanes, whose average loads are issued with the state's.
#pragma once
#include "kernels.hpp"

namespace dgsrhd {

struct LimArgs {
  double* U;             // stage output, limited in place
  const double* avg;     // [NV][nelem] averages of U (written by the stage launch)
  double* Wout;          // the next stage's primitives (written by the stage launch), or null
  double xi[kMaxN1];     // reference nodes on [-1, 1]
  double inv_den;        // 1 / sum_n w_n xi_{d,n}^2 (the same for every d)
  int phys;
  MeshArgs m;
  Tables t;
  PhysParams q;
  Counters* cnt;
};

template <int DIM, int P>
__device__ __forceinline__ double node_weight(const Tables& t, int node) {
  constexpr int N1 = P + 1;
  double wn = t.w[node_coord<N1>(node, 0)];
  if (DIM > 1) wn *= t.w[node_coord<N1>(node, 1)];
  if (DIM > 2) wn *= t.w[node_coord<N1>(node, 2)];
  return wn;
}

__device__ __forceinline__ double minmod3(double a, double b, double c) {
  const bool same = (a > 0.0 && b > 0.0 && c > 0.0) || (a < 0.0 && b < 0.0 && c < 0.0);
  const double mag = fmin(fmin(fabs(a), fabs(b)), fabs(c));
  return same ? copysign(mag, a) : 0.0;
}

// node mirrored along d (coordinate c -> N1 - 1 - c)
template <int DIM, int N1>
__device__ __forceinline__ int mirror_node(int node, int d) {
  const int c = node_coord<N1>(node, d);
  const int stride = d == 0 ? 1 : (d == 1 ? N1 : N1 * N1);
  return node + (N1 - 1 - 2 * c) * stride;
}

constexpr double kLimEps = 1e-10;

// neighbour of element (x, y, z) along d on side dir, or the element itself at a
// non-periodic end
// (selects rather than arrays indexed by the per-lane direction, which could go to scratch)
__device__ __forceinline__ int neighbour_or_self(const MeshArgs& m, int cx, int cy, int cz, int e, int d, int dir) {
  const int n = d == 0 ? m.nex : (d == 1 ? m.ney : m.nez);
  const int stride = d == 0 ? 1 : (d == 1 ? m.nex : m.nex * m.ney);
  const int per = d == 0 ? m.periodic[0] : (d == 1 ? m.periodic[1] : m.periodic[2]);
  const int k = (d == 0 ? cx : (d == 1 ? cy : cz)) + dir;
  if (k < 0) return per ? e + (n - 1) * stride : e;
  if (k >= n) return per ? e - (n - 1) * stride : e;
  return e + dir * stride;
}

template <int DIM, int P>
struct LimGeo {
  using G = Geo<DIM, P>;
  static constexpr int NPE = G::NPE, NV = G::NV, N1 = G::N1;
  static constexpr int EPW = 64 / NPE;  // whole elements per wave
  static constexpr int NT = 256;        // four waves
  static constexpr int EPB = 4 * EPW;   // elements per workgroup
  static constexpr int NS = DIM * NV;   // (direction, component) pairs per element
};

template <int DIM, int P, int EOS>
__global__ __launch_bounds__(256) void k_limit(LimArgs a) {
  using L = LimGeo<DIM, P>;
  constexpr int NV = L::NV, NPE = L::NPE, NT = L::NT, EPW = L::EPW, EPB = L::EPB, N1 = L::N1, NS = L::NS;
  constexpr int KP = (NS + NPE - 1) / NPE;   // pairs per lane
  __shared__ double sbuf[NV * NT];
  __shared__ double sratio[EPB * NS];
  __shared__ int sflag[NT];
  const MeshArgs& m = a.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int ew = lane / NPE, node = lane % NPE;
  const bool lane_ok = ew < EPW;
  const int el = (tid >> 6) * EPW + ew;  // element of the workgroup (lane_ok lanes)
  const int base = tid - node;           // LDS slot of the element's node 0
  // XCD-aware order: each XCD takes a contiguous range of element groups, so the rows
  // of neighbour averages a group gathers are mostly in that XCD's L2 already
  const long long e = (long long)xcd_tile(blockIdx.x, gridDim.x) * EPB + el;
  const bool act = lane_ok && e < m.nelem;
  const long long g = e * NPE + node;
  const long long ne = m.nelem;
  double u[NV], u0[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = u0[v] = act ? a.U[v * m.ntot + g] : 1.0;
  // the density the stage launch recovered (NaN where its recovery failed), loaded with U
  const double rho_stage = (act && a.Wout) ? a.Wout[g] : 0.0;
  // this lane's pairs: own and neighbour averages, and the element's energy scale
  double ub[KP], up[KP], um[KP];
  double E = 0.0;
  if (act) {
    const int ie = (int)e;
    const int cx = ie % m.nex, cy = (ie / m.nex) % m.ney, cz = ie / (m.nex * m.ney);
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const int k = node + j * NPE;
      ub[j] = up[j] = um[j] = 0.0;
      if (k < NS) {
        const int d = k / NV, v = k % NV;
        const double* av = a.avg + v * ne;
        ub[j] = av[e];
        up[j] = av[neighbour_or_self(m, cx, cy, cz, ie, d, +1)];
        um[j] = av[neighbour_or_self(m, cx, cy, cz, ie, d, -1)];
      }
    }
    if (node < NS) E = fabs(a.avg[(NV - 1) * ne + e] + a.avg[e] * a.q.c2);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) sbuf[v * NT + tid] = u[v];
  wave_sync();
  // slope of each pair from the odd parts of the mirror pairs of nodes, minmod bound, ratio
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int k = node + j * NPE;
    if (lane_ok && k < NS) {
      double ratio = 1.0;
      if (act) {
        const int d = k / NV, v = k % NV;
        const double* row = sbuf + v * NT + base;
        double acc = 0.0;
        for (int n = 0; n < NPE; ++n) {
          const double wx = node_weight<DIM, P>(a.t, n) * a.xi[node_coord<N1>(n, d)];
          acc += wx * (0.5 * (row[n] - row[mirror_node<DIM, N1>(n, d)]));
        }
        const double s = acc * a.inv_den;
        const double sl = minmod3(s, up[j] - ub[j], ub[j] - um[j]);
        const double sig = v == 0 ? E * a.q.inv_c2 : (v == NV - 1 ? E : E * a.q.inv_c);
        if (fabs(s - sl) > kLimEps * sig) ratio = sl / s;
      }
      sratio[el * NS + k] = ratio;
    }
  }
  wave_sync();
  double th = 1.0;
  if (act) {
#pragma unroll
    for (int k = 0; k < NS; ++k) th = fmin(th, sratio[el * NS + k]);
  }
  const bool lim = act && th < 1.0;
  count_wave(&counter_slot(a.cnt)->limited, lim && node == 0);
  if (lim) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double avv = a.avg[v * ne + e];
      u[v] = avv + th * (u[v] - avv);
    }
  }
  // (sbuf is rewritten by the operator only after every lane of the wave has read its
  // slopes: the reads above precede the ratio exchange's ordering point)
  if (a.phys) physicality_wave<DIM, P, NT>(u, act, tid, base, node, a.t, a.q, counter_slot(a.cnt), sbuf, sflag);
  if (!act) return;
  // only the nodes the limiter or the operator changed are written (NaN compares unequal)
  bool changed = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) changed = changed || !(u[v] == u0[v]);
  if (changed) {
#pragma unroll
    for (int v = 0; v < NV; ++v) a.U[v * m.ntot + g] = u[v];
  }
  if (a.Wout) {
    // the stage launch recovered every node; recover again (and count) the changed nodes,
    // Newton started from the stage's primitives, and the nodes whose recovery failed
    // there (marked by a NaN density), from the usual start
    const bool marked = !(rho_stage == rho_stage);
    if (changed || marked) {
      double w[NV], wp[NV];
      if (!marked) {
#pragma unroll
        for (int v = 0; v < NV; ++v) wp[v] = a.Wout[v * m.ntot + g];
      }
      // (two calls rather than one through a selected pointer, which would put the start
      // in scratch memory)
      const int st = marked ? con2prim<EOS, DIM>(u, w, a.q) : con2prim<EOS, DIM>(u, w, a.q, wp);
      count_c2p(counter_slot(a.cnt), st, e);
#pragma unroll
      for (int v = 0; v < NV; ++v) a.Wout[v * m.ntot + g] = w[v];
    }
  }
}

}  // namespace dgsrhd
