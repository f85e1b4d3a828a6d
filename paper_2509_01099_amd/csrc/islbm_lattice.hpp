// Device-side lattice descriptions and the MRT collision, in deviation form.
//
// Velocity sets and moment bases follow the double-distribution MRT model of
// Sec. 2.1: D2Q9 / D3Q19 for the flow populations f with Guo's forcing, and
// D2Q5 / D3Q7 for the temperature populations g.  The moment matrices are
// the orthogonal polynomial bases whose action on the second-order
// equilibrium gives the printed equilibrium moments (D2Q9 and D3Q19
// equations of Sec. 2.1); the thermal bases give the printed n^eq.
//
// Populations are handled as deviations d_i = f_i - w_i (flow; w_i the
// lattice weights, i.e. the rest state rho = 1, u = 0) and g_i (thermal; rest
// state 0).  Since M is linear, the collision m+ = m - S(m - m^eq) +
// (I - S/2) M F~ holds for deviation moments with m^eq replaced by
// m^eq(rho, u) - m^eq(1, 0).  Every moment row of these bases is either even
// or odd under e -> -e, so the transforms are evaluated on the pair sums and
// differences d_i +/- d_opp(i), halving the arithmetic; the inverse uses
// M^-1 = M^T diag(1/|M_r|^2) (the rows are orthogonal).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace islbm {

template <typename R>
struct Rates {
  R s_e, s_eps, s_q, s_nu, s_pi, s_m;  // flow rates (D2Q9 uses s_e, s_eps, s_q, s_nu)
  R q_j, q_e, q_nu;                     // thermal rates
  R aT;                                 // thermal equilibrium coefficient a_T
  R gbeta, T0;                          // buoyancy: F_y = rho g beta (T - T0)
};

// ---------------------------------------------------------------------------
// Velocity sets.  Ordering: rest first, then opposite pairs.
// ---------------------------------------------------------------------------
struct D2Q9 {
  static constexpr int Q = 9, D = 2, NP = 4;  // NP opposite pairs
  __host__ __device__ static constexpr int e(int i, int a) {
    constexpr int t[9][3] = {{0, 0, 0}, {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                             {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    return t[i][a];
  }
  // first member of pair k and its opposite
  __host__ __device__ static constexpr int pa(int k) { constexpr int t[4] = {1, 2, 5, 6}; return t[k]; }
  __host__ __device__ static constexpr int pb(int k) { constexpr int t[4] = {3, 4, 7, 8}; return t[k]; }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  // rows: rho, e, eps, jx, qx, jy, qy, pxx, pxy
  __host__ __device__ static constexpr int M(int r, int i) {
    const int x = e(i, 0), y = e(i, 1), s = x * x + y * y;
    switch (r) {
      case 0: return 1;
      case 1: return 3 * s - 4;
      case 2: return (9 * s * s - 21 * s + 8) / 2;
      case 3: return x;
      case 4: return (3 * s - 5) * x;
      case 5: return y;
      case 6: return (3 * s - 5) * y;
      case 7: return x * x - y * y;
      default: return x * y;
    }
  }
};

struct D2Q5 {
  static constexpr int Q = 5, D = 2, NP = 2;
  __host__ __device__ static constexpr int e(int i, int a) {
    constexpr int t[5][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}};
    return t[i][a];
  }
  __host__ __device__ static constexpr int pa(int k) { constexpr int t[2] = {1, 2}; return t[k]; }
  __host__ __device__ static constexpr int pb(int k) { constexpr int t[2] = {3, 4}; return t[k]; }
  // rows: T, jx, jy, 5|e|^2 - 4, ex^2 - ey^2
  __host__ __device__ static constexpr int M(int r, int i) {
    const int x = e(i, 0), y = e(i, 1), s = x * x + y * y;
    switch (r) {
      case 0: return 1;
      case 1: return x;
      case 2: return y;
      case 3: return 5 * s - 4;
      default: return x * x - y * y;
    }
  }
};

struct D3Q19 {
  static constexpr int Q = 19, D = 3, NP = 9;
  __host__ __device__ static constexpr int e(int i, int a) {
    constexpr int t[19][3] = {{0, 0, 0},   {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},   {0, 0, -1}, {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0},  {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    return t[i][a];
  }
  __host__ __device__ static constexpr int pa(int k) { return 2 * k + 1; }
  __host__ __device__ static constexpr int pb(int k) { return 2 * k + 2; }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  // rows: rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz,
  //       pxz, mx, my, mz
  __host__ __device__ static constexpr int M(int r, int i) {
    const int x = e(i, 0), y = e(i, 1), z = e(i, 2);
    const int xx = x * x, yy = y * y, zz = z * z, s = xx + yy + zz;
    switch (r) {
      case 0: return 1;
      case 1: return 19 * s - 30;
      case 2: return (21 * s * s - 53 * s + 24) / 2;
      case 3: return x;
      case 4: return (5 * s - 9) * x;
      case 5: return y;
      case 6: return (5 * s - 9) * y;
      case 7: return z;
      case 8: return (5 * s - 9) * z;
      case 9: return 3 * xx - s;
      case 10: return (3 * s - 5) * (3 * xx - s);
      case 11: return yy - zz;
      case 12: return (3 * s - 5) * (yy - zz);
      case 13: return x * y;
      case 14: return y * z;
      case 15: return x * z;
      case 16: return (yy - zz) * x;
      case 17: return (zz - xx) * y;
      default: return (xx - yy) * z;
    }
  }
};

struct D3Q7 {
  static constexpr int Q = 7, D = 3, NP = 3;
  __host__ __device__ static constexpr int e(int i, int a) {
    constexpr int t[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                             {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    return t[i][a];
  }
  __host__ __device__ static constexpr int pa(int k) { return 2 * k + 1; }
  __host__ __device__ static constexpr int pb(int k) { return 2 * k + 2; }
  // rows: T, jx, jy, jz, 7|e|^2 - 6, 2ex^2 - ey^2 - ez^2, ey^2 - ez^2
  __host__ __device__ static constexpr int M(int r, int i) {
    const int x = e(i, 0), y = e(i, 1), z = e(i, 2), s = x * x + y * y + z * z;
    switch (r) {
      case 0: return 1;
      case 1: return x;
      case 2: return y;
      case 3: return z;
      case 4: return 7 * s - 6;
      case 5: return 2 * x * x - y * y - z * z;
      default: return y * y - z * z;
    }
  }
};

template <class L>
__host__ __device__ constexpr int opp(int i) {
  for (int k = 0; k < L::Q; ++k)
    if (L::e(k, 0) == -L::e(i, 0) && L::e(k, 1) == -L::e(i, 1) && L::e(k, 2) == -L::e(i, 2))
      return k;
  return -1;
}

template <class L>
__host__ __device__ constexpr int norm2(int r) {
  int s = 0;
  for (int i = 0; i < L::Q; ++i) s += L::M(r, i) * L::M(r, i);
  return s;
}

// Row parity under e -> -e: +1 even (depends on pair sums), -1 odd (pair
// differences only), 0 neither (never the case for these bases).
template <class L>
__host__ __device__ constexpr int parity(int r) {
  bool even = true, odd = L::M(r, 0) == 0;
  for (int k = 0; k < L::NP; ++k) {
    if (L::M(r, L::pa(k)) != L::M(r, L::pb(k))) even = false;
    if (L::M(r, L::pa(k)) != -L::M(r, L::pb(k))) odd = false;
  }
  return even ? 1 : (odd ? -1 : 0);
}

template <class L>
__host__ __device__ constexpr bool well_formed() {
  for (int k = 0; k < L::NP; ++k)
    if (opp<L>(L::pa(k)) != L::pb(k)) return false;
  for (int r = 0; r < L::Q; ++r) {
    if (parity<L>(r) == 0) return false;
    for (int c = 0; c < r; ++c) {  // orthogonal rows
      int dot = 0;
      for (int i = 0; i < L::Q; ++i) dot += L::M(r, i) * L::M(c, i);
      if (dot != 0) return false;
    }
  }
  return true;
}
static_assert(well_formed<D2Q9>() && well_formed<D2Q5>() && well_formed<D3Q19>() &&
                  well_formed<D3Q7>(),
              "velocity pairs and orthogonal moment rows");

// acc + c * x for a compile-time integer c; zero terms vanish.
template <int C, typename R>
__device__ __forceinline__ R axpy(R acc, R x) {
  if constexpr (C == 0) return acc;
  else if constexpr (C == 1) return acc + x;
  else if constexpr (C == -1) return acc - x;
  else return acc + R(C) * x;
}

// Moment r from the rest value d0 and pair sums S / differences A.
template <class L, int r, typename R, int... K>
__device__ __forceinline__ R moment(R d0, const R* S, const R* A, std::integer_sequence<int, K...>) {
  R acc = R(0);
  if constexpr (parity<L>(r) == 1) {
    acc = axpy<L::M(r, 0)>(acc, d0);
    ((acc = axpy<L::M(r, L::pa(K))>(acc, S[K])), ...);
  } else {
    ((acc = axpy<L::M(r, L::pa(K))>(acc, A[K])), ...);
  }
  return acc;
}

template <class L, typename R, int... Rw>
__device__ __forceinline__ void forward(const R* d, R* m, std::integer_sequence<int, Rw...>) {
  R S[L::NP], A[L::NP];
#pragma unroll
  for (int k = 0; k < L::NP; ++k) {
    S[k] = d[L::pa(k)] + d[L::pb(k)];
    A[k] = d[L::pa(k)] - d[L::pb(k)];
  }
  ((m[Rw] = moment<L, Rw>(d[0], S, A, std::make_integer_sequence<int, L::NP>{})), ...);
}

// Even / odd part of population pa(k) from scaled moments mn[r] = m[r]/|M_r|^2.
template <class L, int k, int sign, typename R, int... Rw>
__device__ __forceinline__ R back_part(const R* mn, std::integer_sequence<int, Rw...>) {
  R acc = R(0);
  ((acc = (parity<L>(Rw) == sign) ? axpy<L::M(Rw, L::pa(k))>(acc, mn[Rw]) : acc), ...);
  return acc;
}

template <class L, int k, typename R>
__device__ __forceinline__ void back_pair(const R* mn, R* d) {
  const R ev = back_part<L, k, 1>(mn, std::make_integer_sequence<int, L::Q>{});
  const R od = back_part<L, k, -1>(mn, std::make_integer_sequence<int, L::Q>{});
  d[L::pa(k)] = ev + od;
  d[L::pb(k)] = ev - od;
}

template <class L, int r, typename R>
__device__ __forceinline__ R rest_part_term(const R* mn, R acc) {
  return axpy<L::M(r, 0)>(acc, mn[r]);
}

template <class L, typename R, int... K, int... Rw>
__device__ __forceinline__ void backward(const R* m, R* d, std::integer_sequence<int, K...>,
                                         std::integer_sequence<int, Rw...>) {
  R mn[L::Q];
  ((mn[Rw] = m[Rw] * R(1.0 / double(norm2<L>(Rw)))), ...);
  R d0 = R(0);
  ((d0 = rest_part_term<L, Rw>(mn, d0)), ...);
  d[0] = d0;
  (back_pair<L, K>(mn, d), ...);
}

template <class L, typename R>
__device__ __forceinline__ void to_moments(const R* d, R* m) {
  forward<L>(d, m, std::make_integer_sequence<int, L::Q>{});
}

template <class L, typename R>
__device__ __forceinline__ void from_moments(const R* m, R* d) {
  backward<L>(m, d, std::make_integer_sequence<int, L::NP>{}, std::make_integer_sequence<int, L::Q>{});
}

// ---------------------------------------------------------------------------
// Macroscopic state of one node, from pre-collision deviation moments.
// ---------------------------------------------------------------------------
template <typename R>
struct Macro {
  R rho, drho, T, Fy;
  R ru[3];  // rho u = j + F/2
  R u[3];
};

// ---------------------------------------------------------------------------
// Relaxation in moment space (deviation form), per lattice pair.
// m: flow moments (in/out), n: thermal moments (in/out).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void relax_2d(R* m, R* n, const Rates<R>& k, Macro<R>& s) {
  s.drho = m[0];
  s.rho = R(1) + s.drho;
  s.T = n[0];
  s.Fy = s.rho * k.gbeta * (s.T - k.T0);
  const R inv = R(1) / s.rho;
  s.ru[0] = m[3];
  s.ru[1] = m[5] + R(0.5) * s.Fy;
  s.ru[2] = R(0);
  s.u[0] = s.ru[0] * inv;
  s.u[1] = s.ru[1] * inv;
  s.u[2] = R(0);
  const R ux = s.u[0], uy = s.u[1];
  const R ru2 = s.ru[0] * ux + s.ru[1] * uy;  // rho |u|^2
  const R uF = uy * s.Fy;
  const R he = R(1) - R(0.5) * k.s_e, hp = R(1) - R(0.5) * k.s_eps;
  const R hq = R(1) - R(0.5) * k.s_q, hn = R(1) - R(0.5) * k.s_nu;
  // m^eq - m^eq(1,0): e = -2 drho + 3 rho u^2, eps = drho - 3 rho u^2,
  // q = -rho u, pxx = rho (u^2 - v^2), pxy = rho u v.  M F~ with F = (0, Fy).
  m[1] = m[1] - k.s_e * (m[1] - (R(-2) * s.drho + R(3) * ru2)) + he * R(6) * uF;
  m[2] = m[2] - k.s_eps * (m[2] - (s.drho - R(3) * ru2)) - hp * R(6) * uF;
  m[3] = m[3];
  m[4] = m[4] - k.s_q * (m[4] + s.ru[0]);
  m[5] = m[5] + s.Fy;
  m[6] = m[6] - k.s_q * (m[6] + s.ru[1]) - hq * s.Fy;
  m[7] = m[7] - k.s_nu * (m[7] - (s.ru[0] * ux - s.ru[1] * uy)) - hn * R(2) * uF;
  m[8] = m[8] - k.s_nu * (m[8] - s.ru[0] * uy) + hn * ux * s.Fy;
  // D2Q5: n^eq = [T, uT, vT, a_T T, 0]
  n[1] = n[1] - k.q_j * (n[1] - ux * s.T);
  n[2] = n[2] - k.q_j * (n[2] - uy * s.T);
  n[3] = n[3] - k.q_e * (n[3] - k.aT * s.T);
  n[4] = n[4] - k.q_nu * n[4];
}

template <typename R>
__device__ __forceinline__ void relax_3d(R* m, R* n, const Rates<R>& k, Macro<R>& s) {
  s.drho = m[0];
  s.rho = R(1) + s.drho;
  s.T = n[0];
  s.Fy = s.rho * k.gbeta * (s.T - k.T0);
  const R inv = R(1) / s.rho;
  s.ru[0] = m[3];
  s.ru[1] = m[5] + R(0.5) * s.Fy;
  s.ru[2] = m[7];
  s.u[0] = s.ru[0] * inv;
  s.u[1] = s.ru[1] * inv;
  s.u[2] = s.ru[2] * inv;
  const R ux = s.u[0], uy = s.u[1], uz = s.u[2];
  const R rxx = s.ru[0] * ux, ryy = s.ru[1] * uy, rzz = s.ru[2] * uz;
  const R ru2 = rxx + ryy + rzz;
  const R uF = uy * s.Fy;
  const R he = R(1) - R(0.5) * k.s_e, hp = R(1) - R(0.5) * k.s_eps;
  const R hq = R(1) - R(0.5) * k.s_q, hn = R(1) - R(0.5) * k.s_nu;
  const R hpi = R(1) - R(0.5) * k.s_pi;
  const R c23 = R(2.0 / 3.0);
  const R pxx = R(2) * rxx - ryy - rzz, pww = ryy - rzz;
  m[1] = m[1] - k.s_e * (m[1] - (R(-11) * s.drho + R(19) * ru2)) + he * R(38) * uF;
  m[2] = m[2] - k.s_eps * (m[2] - (R(3) * s.drho - R(5.5) * ru2)) - hp * R(11) * uF;
  m[4] = m[4] - k.s_q * (m[4] + c23 * s.ru[0]);
  m[5] = m[5] + s.Fy;
  m[6] = m[6] - k.s_q * (m[6] + c23 * s.ru[1]) - hq * c23 * s.Fy;
  m[8] = m[8] - k.s_q * (m[8] + c23 * s.ru[2]);
  m[9] = m[9] - k.s_nu * (m[9] - pxx) - hn * R(2) * uF;
  m[10] = m[10] - k.s_pi * (m[10] + R(0.5) * pxx) + hpi * uF;
  m[11] = m[11] - k.s_nu * (m[11] - pww) + hn * R(2) * uF;
  m[12] = m[12] - k.s_pi * (m[12] + R(0.5) * pww) - hpi * uF;
  m[13] = m[13] - k.s_nu * (m[13] - s.ru[0] * uy) + hn * ux * s.Fy;
  m[14] = m[14] - k.s_nu * (m[14] - s.ru[1] * uz) + hn * uz * s.Fy;
  m[15] = m[15] - k.s_nu * (m[15] - s.ru[0] * uz);
  m[16] = m[16] - k.s_m * m[16];
  m[17] = m[17] - k.s_m * m[17];
  m[18] = m[18] - k.s_m * m[18];
  // D3Q7: n^eq = [T, uT, vT, wT, a_T T, 0, 0]
  n[1] = n[1] - k.q_j * (n[1] - ux * s.T);
  n[2] = n[2] - k.q_j * (n[2] - uy * s.T);
  n[3] = n[3] - k.q_j * (n[3] - uz * s.T);
  n[4] = n[4] - k.q_e * (n[4] - k.aT * s.T);
  n[5] = n[5] - k.q_nu * n[5];
  n[6] = n[6] - k.q_nu * n[6];
}

template <int D>
struct Pair;
template <>
struct Pair<2> {
  using F = D2Q9;
  using G = D2Q5;
};
template <>
struct Pair<3> {
  using F = D3Q19;
  using G = D3Q7;
};

// Full collision of one node: d (flow deviations) and g in, post-collision
// values out (in place); s receives the macroscopic state.
template <int D, typename R>
__device__ __forceinline__ void collide(R* d, R* g, const Rates<R>& k, Macro<R>& s) {
  using LF = typename Pair<D>::F;
  using LG = typename Pair<D>::G;
  R m[LF::Q], n[LG::Q];
  to_moments<LF>(d, m);
  to_moments<LG>(g, n);
  if constexpr (D == 2) relax_2d(m, n, k, s);
  else relax_3d(m, n, k, s);
  from_moments<LF>(m, d);
  from_moments<LG>(n, g);
}

// Macroscopic state from post-collision deviations (rho and T are invariant
// under collision; the momentum of f+ is j + F, so rho u = j+ - F/2).
template <int D, typename R>
__device__ __forceinline__ void macro_post(const R* d, const R* g, const Rates<R>& k, Macro<R>& s) {
  using LF = typename Pair<D>::F;
  using LG = typename Pair<D>::G;
  R drho = R(0), T = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < LF::Q; ++i) {
    drho += d[i];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (LF::e(i, a) != 0) j[a] += R(LF::e(i, a)) * d[i];
  }
#pragma unroll
  for (int i = 0; i < LG::Q; ++i) T += g[i];
  s.drho = drho;
  s.rho = R(1) + drho;
  s.T = T;
  s.Fy = s.rho * k.gbeta * (T - k.T0);
  s.ru[0] = j[0];
  s.ru[1] = j[1] - R(0.5) * s.Fy;
  s.ru[2] = j[2];
  const R inv = R(1) / s.rho;
  for (int a = 0; a < 3; ++a) s.u[a] = s.ru[a] * inv;
}

}  // namespace islbm
