// Slope limiter for basis orders >= 1 (Sec. 2.3 names the minmod limiter of van Leer
// 1979 and the scaling limiter of Moe, Rossmanith & Seal 2015 for the p >= 1 shock
// runs): minmod-bounded slopes applied as one scaling factor per element.
//
// k_avg     element averages of every component, [var][element], one element per
//           group of NPE lanes (the quadrature sum in node order).
// k_limit   per element: for each component k and direction d the slope s, the
//           coefficient of xi_d in the element's Legendre expansion (sum_n w_n
//           xi_{d,n} u_n / sum_n w_n xi_{d,n}^2, mirror nodes paired so that a constant
//           element has slope exactly 0), and its bound s~ = minmod(s, ubar_+ - ubar,
//           ubar - ubar_-) by the neighbours' averages (periodic wrap, the element's
//           own average at a non-periodic end); theta = the least s~ / s over the pairs
//           where |s - s~| exceeds kLimEps times the component's scale (the average
//           energy E = |tau + D c^2| over c^2 for D, over c for S, E for tau); where
//           theta < 1 every node moves to ubar + theta (u - ubar).  Then the
//           physicality operator (Sec. 2.5) and the recovery of the next stage's
//           primitives, all before one write of U and W.  One factor for all
//           components keeps every node on the segment to the (admissible) average.
//
// Both kernels use the workgroup layout of the operator kernel: EPB consecutive
// elements per workgroup, one node per lane.
#pragma once
#include "kernels.hpp"

namespace dgsrhd {

struct LimArgs {
  double* U;             // stage output, limited in place
  const double* avg;     // [NV][nelem] averages of U (k_avg)
  double* Wout;          // primitives of the limited state, or null
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

template <int DIM, int P>
__global__ __launch_bounds__((Geo<DIM, P>::NT)) void k_avg(const double* __restrict__ U, double* __restrict__ avg,
                                                         MeshArgs m, Tables t) {
  using G = Geo<DIM, P>;
  constexpr int NV = G::NV, NPE = G::NPE, NT = G::NT, EPB = G::EPB;
  __shared__ double sbuf[NV * NT];
  const int tid = threadIdx.x;
  const int el = tid / NPE, node = tid % NPE;
  const long long e = (long long)blockIdx.x * EPB + el;
  const bool act = e < m.nelem;
  const long long g = e * NPE + node;
  const double wn = node_weight<DIM, P>(t, node);
#pragma unroll
  for (int v = 0; v < NV; ++v) sbuf[v * NT + tid] = act ? wn * U[v * m.ntot + g] : 0.0;
  __syncthreads();
  if (!act) return;
  for (int v = node; v < NV; v += NPE) {
    double acc = 0.0;
    for (int n = 0; n < NPE; ++n) acc += sbuf[v * NT + el * NPE + n];
    avg[(long long)v * m.nelem + e] = acc * t.inv_wsum;
  }
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

template <int DIM, int P, int EOS>
__global__ __launch_bounds__((Geo<DIM, P>::NT)) void k_limit(LimArgs a) {
  using G = Geo<DIM, P>;
  constexpr int NV = G::NV, NPE = G::NPE, NT = G::NT, EPB = G::EPB, N1 = G::N1;
  constexpr int NS = DIM * NV;  // (direction, component) pairs per element
  __shared__ double sbuf[NV * NT];
  __shared__ double sterm[NS * NT];
  __shared__ double sratio[EPB * NS];
  __shared__ int sflag[NT];
  __shared__ int svote[(NT + 63) / 64];
  const MeshArgs& m = a.m;
  const int tid = threadIdx.x;
  const int el = tid / NPE, node = tid % NPE;
  const long long e = (long long)blockIdx.x * EPB + el;
  const bool act = e < m.nelem;
  const long long g = e * NPE + node;
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    u[v] = act ? a.U[v * m.ntot + g] : 1.0;
    sbuf[v * NT + tid] = u[v];
  }
  __syncthreads();
  // odd part of each mirror pair times w_n xi_{d,n}
  const double wn = node_weight<DIM, P>(a.t, node);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int mn = el * NPE + mirror_node<DIM, N1>(node, d);
    const double wx = wn * a.xi[node_coord<N1>(node, d)];
#pragma unroll
    for (int v = 0; v < NV; ++v) sterm[(d * NV + v) * NT + tid] = wx * (0.5 * (u[v] - sbuf[v * NT + mn]));
  }
  __syncthreads();
  // one lane per (d, v) pair: slope, minmod bound, ratio
  for (int k = node; k < NS; k += NPE) {
    double ratio = 1.0;
    if (act) {
      const int d = k / NV, v = k % NV;
      double acc = 0.0;
      for (int n = 0; n < NPE; ++n) acc += sterm[k * NT + el * NPE + n];
      const double s = acc * a.inv_den;
      const double* av = a.avg + (long long)v * m.nelem;
      const double ub = av[e];
      const int ep = neighbour(m, (int)e, d, +1), em = neighbour(m, (int)e, d, -1);
      const double fwd = (ep < 0 ? ub : av[ep]) - ub;
      const double bwd = ub - (em < 0 ? ub : av[em]);
      const double sl = minmod3(s, fwd, bwd);
      const double E = fabs(a.avg[(long long)(NV - 1) * m.nelem + e] + a.avg[e] * a.q.c2);
      const double sig = v == 0 ? E * a.q.inv_c2 : (v == NV - 1 ? E : E * a.q.inv_c);
      if (fabs(s - sl) > kLimEps * sig) ratio = sl / s;
    }
    sratio[el * NS + k] = ratio;
  }
  __syncthreads();
  double th = 1.0;
  for (int k = 0; k < NS; ++k) th = fmin(th, sratio[el * NS + k]);
  const bool lim = act && th < 1.0;
  count_wave(&counter_slot(a.cnt)->limited, lim && node == 0);
  if (lim) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double ub = a.avg[(long long)v * m.nelem + e];
      u[v] = ub + th * (u[v] - ub);
    }
  }
  if (a.phys) physicality_block_t<DIM, P, NT>(u, act, tid, el, node, a.t, a.q, counter_slot(a.cnt), sbuf, sflag, svote);
  if (!act) return;
#pragma unroll
  for (int v = 0; v < NV; ++v) a.U[v * m.ntot + g] = u[v];
  if (a.Wout) {
    double w[NV];
    const int st = con2prim<EOS, DIM>(u, w, a.q);
    count_c2p(counter_slot(a.cnt), st, e);
#pragma unroll
    for (int v = 0; v < NV; ++v) a.Wout[v * m.ntot + g] = w[v];
  }
}

}  // namespace dgsrhd
