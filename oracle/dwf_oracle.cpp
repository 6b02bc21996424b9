// FP64 CPU oracle for the domain-wall Dirac operator and its CG solve.
//
// TEST INFRASTRUCTURE ONLY. This file is called by the test suite, the
// smoke check and the CPU-baseline leg of the benchmark. The product library
// never links or calls it, and it shares no code, header or table with the
// HIP path.
//
// It is written for reading, not for speed: plain loops over lattice
// coordinates, explicit 4x4 gamma matrices applied by matrix-vector products,
// std::complex<double> arithmetic, compiled with -ffp-contract=off, and M_ee^-1
// by dense LU of the (4 Ls) x (4 Ls) spin-by-s block of M_ee at a 4D site.
//
// What the paper fixes, and what the code below takes as its definition:
// * The paper (Sections 4.1-4.3) names the Domain Wall kernel -- the 4D Wilson
//   hopping term with SU(3) link multiplies applied on every slice of the fifth
//   dimension -- as the kernel whose speed it measures (Section 4.1), and
//   counts 1320 real flops per 5D site update for it (Table 3).
// * The paper writes neither the operator nor a solver as formulas, so the
//   standard lattice-QCD conventions below are the reading taken (each is
//   pinned by a closed form, an invariant or brute force in the CPU tests):
//     - lattice coordinates (x,y,z,t), lex = ((t*Lz+z)*Ly+y)*Lx+x;
//     - boundary factor bc[mu] (+1 periodic, -1 antiperiodic) multiplies every
//       hop that crosses the mu boundary;
//     - DeGrand-Rossi chiral gamma basis, gamma5 = gx*gy*gz*gt = diag(1,1,-1,-1);
//     - hop: (D_h psi)(x) = sum_mu [ (1-g_mu) U_mu(x) psi(x+mu)
//                                  + (1+g_mu) U_mu(x-mu)^dag psi(x-mu) ];
//       its adjoint swaps (1-g_mu) and (1+g_mu);
//     - Wilson operator at mass -M5: D_W = (4-M5) - D_h/2;
//     - fifth dimension: S_u psi_s = psi_{s+1} (row Ls-1 takes -mf psi_0),
//       S_d psi_s = psi_{s-1} (row 0 takes -mf psi_{Ls-1}),
//       C = P- S_u + P+ S_d with P+- = (1 +- g5)/2, A = b + c C, B = 1 - C;
//     - Mobius domain-wall operator D = D_W A + B (Shamir: b=1, c=0), and its
//       adjoint D^dag = A^dag D_W^dag + B^dag;
//     - 4D even-odd blocks: M_ee = M_oo = the 4D-local part of D,
//       M_pq = -1/2 P_p D_h A P_q for p != q, Schur complement on odd sites
//       M_pc = M_oo - M_oe M_ee^-1 M_eo;
//     - CG (Hestenes-Stiefel) on M_pc^dag M_pc from x0 = 0.
//
// Field layouts (interleaved complex128):
//   U[mu][lex][a][b], psi[s][lex][spin][colour].
#include <complex>
#include <cstdint>
#include <cstring>
#include <cmath>
#include <vector>

typedef std::complex<double> cd;

namespace {

struct Action {
  int32_t L[4];
  int32_t Ls;
  int32_t bc[4];
  double M5, mf, b, c;
};

struct Gammas {
  cd g[4][4][4];  // g[mu][row][col]
  cd g5[4][4];
  cd Pp[4][4];    // (1 + g5)/2
  cd Pm[4][4];    // (1 - g5)/2
  Gammas() {
    const cd i(0.0, 1.0);
    std::memset((void*)g, 0, sizeof(g));
    // gamma_x
    g[0][0][3] = i;  g[0][1][2] = i;  g[0][2][1] = -i; g[0][3][0] = -i;
    // gamma_y
    g[1][0][3] = -1; g[1][1][2] = 1;  g[1][2][1] = 1;  g[1][3][0] = -1;
    // gamma_z
    g[2][0][2] = i;  g[2][1][3] = -i; g[2][2][0] = -i; g[2][3][1] = i;
    // gamma_t
    g[3][0][2] = 1;  g[3][1][3] = 1;  g[3][2][0] = 1;  g[3][3][1] = 1;
    // gamma5 = gx gy gz gt, computed by matrix products
    cd t1[4][4], t2[4][4];
    matmul(g[0], g[1], t1);
    matmul(t1, g[2], t2);
    matmul(t2, g[3], g5);
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        const double id = (r == c) ? 1.0 : 0.0;
        Pp[r][c] = 0.5 * (id + g5[r][c]);
        Pm[r][c] = 0.5 * (id - g5[r][c]);
      }
  }
  static void matmul(const cd a[4][4], const cd b[4][4], cd out[4][4]) {
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        cd acc = 0;
        for (int k = 0; k < 4; ++k) acc += a[r][k] * b[k][c];
        out[r][c] = acc;
      }
  }
};

const Gammas& gam() {
  static Gammas G;
  return G;
}

inline long volume(const Action& a) {
  return (long)a.L[0] * a.L[1] * a.L[2] * a.L[3];
}

inline void coords(const Action& a, long lex, int x[4]) {
  for (int mu = 0; mu < 4; ++mu) {
    x[mu] = (int)(lex % a.L[mu]);
    lex /= a.L[mu];
  }
}

inline long lexof(const Action& a, const int x[4]) {
  return (((long)x[3] * a.L[2] + x[2]) * a.L[1] + x[1]) * a.L[0] + x[0];
}

inline int parity_of(const int x[4]) { return (x[0] + x[1] + x[2] + x[3]) & 1; }

inline const cd* link(const cd* U, long V, int mu, long lex) { return U + ((long)mu * V + lex) * 9; }
inline const cd* spin_at(const cd* f, long V, int s, long lex) { return f + ((long)s * V + lex) * 12; }
inline cd* spin_at(cd* f, long V, int s, long lex) { return f + ((long)s * V + lex) * 12; }

// v[spin][a] = sum_b M[a][b] w[spin][b], M = U or U^dag
inline void colour_mul(const cd* U, bool dag, const cd* w, cd* v) {
  for (int sp = 0; sp < 4; ++sp)
    for (int a = 0; a < 3; ++a) {
      cd acc = 0;
      for (int b = 0; b < 3; ++b) {
        const cd m = dag ? std::conj(U[b * 3 + a]) : U[a * 3 + b];
        acc += m * w[sp * 3 + b];
      }
      v[sp * 3 + a] = acc;
    }
}

// acc[alpha][a] += fac * sum_beta (1 + sgn*g_mu)[alpha][beta] v[beta][a]
inline void spin_proj_acc(int mu, int sgn, cd fac, const cd* v, cd* acc) {
  const Gammas& G = gam();
  for (int al = 0; al < 4; ++al)
    for (int a = 0; a < 3; ++a) {
      cd t = 0;
      for (int be = 0; be < 4; ++be) {
        const cd m = (al == be ? 1.0 : 0.0) + (double)sgn * G.g[mu][al][be];
        t += m * v[be * 3 + a];
      }
      acc[al * 3 + a] += fac * t;
    }
}

// (D_h f)(x,s) or (D_h^dag f)(x,s) at one 5D site; result in out[12]. The
// input field is read through get(s, lex, w[12]) so that callers can supply
// either a stored field or values formed on the fly.
template <class Get>
void hop_site_fn(const Action& a, const cd* U, Get get, int s, long lex, int dagger, cd* out) {
  const long V = volume(a);
  int x[4];
  coords(a, lex, x);
  for (int k = 0; k < 12; ++k) out[k] = 0;
  cd v[12], w[12];
  const int fsgn = dagger ? +1 : -1;  // forward hop uses (1 + fsgn*g_mu)
  for (int mu = 0; mu < 4; ++mu) {
    // forward neighbour x + mu
    int y[4] = {x[0], x[1], x[2], x[3]};
    double eta = 1.0;
    y[mu] = x[mu] + 1;
    if (y[mu] == a.L[mu]) { y[mu] = 0; eta = a.bc[mu]; }
    get(s, lexof(a, y), w);
    colour_mul(link(U, V, mu, lex), false, w, v);
    spin_proj_acc(mu, fsgn, cd(eta, 0), v, out);
    // backward neighbour x - mu
    int z[4] = {x[0], x[1], x[2], x[3]};
    eta = 1.0;
    z[mu] = x[mu] - 1;
    if (z[mu] < 0) { z[mu] = a.L[mu] - 1; eta = a.bc[mu]; }
    const long zl = lexof(a, z);
    get(s, zl, w);
    colour_mul(link(U, V, mu, zl), true, w, v);
    spin_proj_acc(mu, -fsgn, cd(eta, 0), v, out);
  }
}

void hop_site(const Action& a, const cd* U, const cd* in, int s, long lex, int dagger, cd* out) {
  const long V = volume(a);
  auto get = [&](int ss, long l, cd* w) {
    const cd* src = spin_at(in, V, ss, l);
    for (int k = 0; k < 12; ++k) w[k] = src[k];
  };
  hop_site_fn(a, U, get, s, lex, dagger, out);
}

// Fifth-dimension shifts at one 5D site: returns (S_u f)(x,s) or (S_d f)(x,s).
inline void shift_up(const Action& a, const cd* f, int s, long lex, cd* out) {
  const long V = volume(a);
  const int sp = s + 1;
  if (sp < a.Ls) {
    const cd* src = spin_at(f, V, sp, lex);
    for (int k = 0; k < 12; ++k) out[k] = src[k];
  } else {
    const cd* src = spin_at(f, V, 0, lex);
    for (int k = 0; k < 12; ++k) out[k] = -a.mf * src[k];
  }
}
inline void shift_dn(const Action& a, const cd* f, int s, long lex, cd* out) {
  const long V = volume(a);
  const int sm = s - 1;
  if (sm >= 0) {
    const cd* src = spin_at(f, V, sm, lex);
    for (int k = 0; k < 12; ++k) out[k] = src[k];
  } else {
    const cd* src = spin_at(f, V, a.Ls - 1, lex);
    for (int k = 0; k < 12; ++k) out[k] = -a.mf * src[k];
  }
}

// out[alpha][a] += fac * sum_beta P[alpha][beta] w[beta][a]
inline void spin_mat_acc(const cd P[4][4], cd fac, const cd* w, cd* out) {
  for (int al = 0; al < 4; ++al)
    for (int a = 0; a < 3; ++a) {
      cd t = 0;
      for (int be = 0; be < 4; ++be) t += P[al][be] * w[be * 3 + a];
      out[al * 3 + a] += fac * t;
    }
}

// (C f)(x,s) (dagger=0) or (C^dag f)(x,s) (dagger=1) at one 5D site.
//   C = P- S_u + P+ S_d,   C^dag = P- S_d + P+ S_u.
void cop_site(const Action& a, const cd* f, int s, long lex, int dagger, cd* out) {
  const Gammas& G = gam();
  cd up[12], dn[12];
  shift_up(a, f, s, lex, up);
  shift_dn(a, f, s, lex, dn);
  for (int k = 0; k < 12; ++k) out[k] = 0;
  if (!dagger) {
    spin_mat_acc(G.Pm, 1.0, up, out);
    spin_mat_acc(G.Pp, 1.0, dn, out);
  } else {
    spin_mat_acc(G.Pm, 1.0, dn, out);
    spin_mat_acc(G.Pp, 1.0, up, out);
  }
}

// out = x0 * f + x1 * (C f) or with C^dag, on every 5D site.
void local_op(const Action& a, const cd* f, cd* out, double x0, double x1, int dagger) {
  const long V = volume(a);
#pragma omp parallel for schedule(static)
  for (long lex = 0; lex < V; ++lex) {
    cd t[12];
    for (int s = 0; s < a.Ls; ++s) {
      cop_site(a, f, s, lex, dagger, t);
      const cd* src = spin_at(f, V, s, lex);
      cd* dst = spin_at(out, V, s, lex);
      for (int k = 0; k < 12; ++k) dst[k] = x0 * src[k] + x1 * t[k];
    }
  }
}

// out(x,s) = D_h (or D_h^dag) in, restricted to sites of parity `par` (-1: all);
// other sites are set to zero.
void hop_field(const Action& a, const cd* U, const cd* in, cd* out, int dagger, int par) {
  const long V = volume(a);
#pragma omp parallel for schedule(static)
  for (long lex = 0; lex < V; ++lex) {
    int x[4];
    coords(a, lex, x);
    const bool on = (par < 0) || (parity_of(x) == par);
    for (int s = 0; s < a.Ls; ++s) {
      cd* dst = spin_at(out, V, s, lex);
      if (on) hop_site(a, U, in, s, lex, dagger, dst);
      else for (int k = 0; k < 12; ++k) dst[k] = 0;
    }
  }
}

void mask_parity(const Action& a, cd* f, int par) {
  const long V = volume(a);
#pragma omp parallel for schedule(static)
  for (long lex = 0; lex < V; ++lex) {
    int x[4];
    coords(a, lex, x);
    if (parity_of(x) != par)
      for (int s = 0; s < a.Ls; ++s) {
        cd* dst = spin_at(f, V, s, lex);
        for (int k = 0; k < 12; ++k) dst[k] = 0;
      }
  }
}

inline double alpha_of(const Action& a) { return a.b * (4.0 - a.M5) + 1.0; }
inline double beta_of(const Action& a) { return a.c * (4.0 - a.M5) - 1.0; }

// ---- dense LU for the 4D-local block of M_ee ------------------------------
struct LU {
  int n;
  std::vector<cd> m;   // row-major, L and U packed
  std::vector<int> piv;
};

// Builds the (4 Ls) x (4 Ls) complex matrix of M_ee (or M_ee^dag) acting on
// index (s, spin) at one 4D site and one colour, then factorises it.
LU factor_mee(const Action& a, int dagger) {
  const Gammas& G = gam();
  const int Ls = a.Ls, n = 4 * Ls;
  const double al = alpha_of(a), be = beta_of(a);
  std::vector<cd> M((size_t)n * n, cd(0));
  auto at = [&](int s, int sp, int t, int tp) -> cd& { return M[(size_t)(s * 4 + sp) * n + (t * 4 + tp)]; };
  // S_u[s][t]: t = s+1, or (Ls-1 -> 0 with -mf); S_d[s][t]: t = s-1, or (0 -> Ls-1 with -mf)
  std::vector<double> Su((size_t)Ls * Ls, 0.0), Sd((size_t)Ls * Ls, 0.0);
  for (int s = 0; s < Ls; ++s) {
    if (s + 1 < Ls) Su[s * Ls + s + 1] = 1.0; else Su[s * Ls + 0] = -a.mf;
    if (s - 1 >= 0) Sd[s * Ls + s - 1] = 1.0; else Sd[s * Ls + Ls - 1] = -a.mf;
  }
  for (int s = 0; s < Ls; ++s)
    for (int t = 0; t < Ls; ++t)
      for (int sp = 0; sp < 4; ++sp)
        for (int tp = 0; tp < 4; ++tp) {
          cd v = (s == t && sp == tp) ? cd(al) : cd(0);
          v += be * (Su[s * Ls + t] * G.Pm[sp][tp] + Sd[s * Ls + t] * G.Pp[sp][tp]);
          at(s, sp, t, tp) = v;
        }
  if (dagger) {
    std::vector<cd> T((size_t)n * n);
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) T[(size_t)r * n + c] = std::conj(M[(size_t)c * n + r]);
    M.swap(T);
  }
  LU lu;
  lu.n = n;
  lu.piv.resize(n);
  // Gaussian elimination with partial pivoting (Doolittle, in place)
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(M[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r) {
      const double v = std::abs(M[(size_t)r * n + k]);
      if (v > best) { best = v; p = r; }
    }
    lu.piv[k] = p;
    if (p != k)
      for (int c = 0; c < n; ++c) std::swap(M[(size_t)k * n + c], M[(size_t)p * n + c]);
    for (int r = k + 1; r < n; ++r) {
      const cd f = M[(size_t)r * n + k] / M[(size_t)k * n + k];
      M[(size_t)r * n + k] = f;
      for (int c = k + 1; c < n; ++c) M[(size_t)r * n + c] -= f * M[(size_t)k * n + c];
    }
  }
  lu.m.swap(M);
  return lu;
}

void lu_solve(const LU& lu, cd* v) {
  const int n = lu.n;
  for (int k = 0; k < n; ++k) std::swap(v[k], v[lu.piv[k]]);
  for (int r = 0; r < n; ++r) {
    cd t = v[r];
    for (int c = 0; c < r; ++c) t -= lu.m[(size_t)r * n + c] * v[c];
    v[r] = t;
  }
  for (int r = n - 1; r >= 0; --r) {
    cd t = v[r];
    for (int c = r + 1; c < n; ++c) t -= lu.m[(size_t)r * n + c] * v[c];
    v[r] = t / lu.m[(size_t)r * n + r];
  }
}

// out = M_ee^-1 in (or M_ee^-dag in) on every 4D site.
void mee_inverse(const Action& a, const cd* in, cd* out, int dagger) {
  const LU lu = factor_mee(a, dagger);
  const long V = volume(a);
  const int Ls = a.Ls;
#pragma omp parallel for schedule(static)
  for (long lex = 0; lex < V; ++lex) {
    std::vector<cd> v((size_t)4 * Ls);
    for (int col = 0; col < 3; ++col) {
      for (int s = 0; s < Ls; ++s)
        for (int sp = 0; sp < 4; ++sp) v[s * 4 + sp] = spin_at(in, V, s, lex)[sp * 3 + col];
      lu_solve(lu, v.data());
      for (int s = 0; s < Ls; ++s)
        for (int sp = 0; sp < 4; ++sp) spin_at(out, V, s, lex)[sp * 3 + col] = v[s * 4 + sp];
    }
  }
}

inline size_t field_len(const Action& a) { return (size_t)volume(a) * a.Ls * 12; }

// Full operator D (dagger=0) or D^dag (dagger=1) on the whole 5D lattice.
void dwf_full(const Action& a, const cd* U, const cd* in, cd* out, int dagger) {
  const size_t n = field_len(a);
  std::vector<cd> t1(n), t2(n);
  if (!dagger) {
    // chi = A in ; out = D_W chi + B in = (4-M5) chi - D_h chi / 2 + in - C in
    local_op(a, in, t1.data(), a.b, a.c, 0);
    hop_field(a, U, t1.data(), t2.data(), 0, -1);
    local_op(a, in, out, 1.0, -1.0, 0);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < (long)n; ++k) out[k] += (4.0 - a.M5) * t1[k] - 0.5 * t2[k];
  } else {
    // w = D_W^dag in ; out = A^dag w + B^dag in
    hop_field(a, U, in, t2.data(), 1, -1);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < (long)n; ++k) t1[k] = (4.0 - a.M5) * in[k] - 0.5 * t2[k];
    local_op(a, t1.data(), t2.data(), a.b, a.c, 1);
    local_op(a, in, out, 1.0, -1.0, 1);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < (long)n; ++k) out[k] += t2[k];
  }
}

// Off-diagonal block. dagger=0: M_{p,q} = -1/2 P_p D_h A P_q.
// dagger=1: (M_{q,p})^dag = -1/2 P_p A^dag D_h^dag P_q. In both cases the input
// lives on parity q = 1-p and the output on parity p.
void deo(const Action& a, const cd* U, const cd* in, cd* out, int p, int dagger) {
  const size_t n = field_len(a);
  std::vector<cd> t1(in, in + n), t2(n);
  mask_parity(a, t1.data(), 1 - p);
  if (!dagger) {
    local_op(a, t1.data(), t2.data(), a.b, a.c, 0);
    hop_field(a, U, t2.data(), out, 0, p);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < (long)n; ++k) out[k] *= -0.5;
  } else {
    hop_field(a, U, t1.data(), t2.data(), 1, p);
    local_op(a, t2.data(), out, a.b, a.c, 1);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < (long)n; ++k) out[k] *= -0.5;
    mask_parity(a, out, p);
  }
}

// M_pc = M_oo - M_oe M_ee^-1 M_eo (dagger=0), or its adjoint, on odd sites.
void mpc(const Action& a, const cd* U, const cd* in, cd* out, int dagger) {
  const size_t n = field_len(a);
  std::vector<cd> x(in, in + n), t1(n), t2(n), t3(n);
  mask_parity(a, x.data(), 1);
  deo(a, U, x.data(), t1.data(), 0, dagger);           // odd -> even
  mee_inverse(a, t1.data(), t2.data(), dagger);         // even
  mask_parity(a, t2.data(), 0);
  deo(a, U, t2.data(), t3.data(), 1, dagger);           // even -> odd
  local_op(a, x.data(), out, alpha_of(a), beta_of(a), dagger);
#pragma omp parallel for schedule(static)
  for (long k = 0; k < (long)n; ++k) out[k] -= t3[k];
  mask_parity(a, out, 1);
}

double dot_re(const cd* u, const cd* v, size_t n) {
  double acc = 0;
  for (size_t k = 0; k < n; ++k) acc += u[k].real() * v[k].real() + u[k].imag() * v[k].imag();
  return acc;
}

}  // namespace

extern "C" {

// The four gamma matrices followed by gamma5, each 4x4 row-major (80 entries).
void or_gammas(cd* out) {
  const Gammas& G = gam();
  for (int mu = 0; mu < 4; ++mu)
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) out[(mu * 4 + r) * 4 + c] = G.g[mu][r][c];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) out[(16 * 4) + r * 4 + c] = G.g5[r][c];
}

// D_h (dagger=0) or D_h^dag (dagger=1) on every 5D site.
void or_hop(const Action* a, const cd* U, const cd* in, cd* out, int dagger) {
  hop_field(*a, U, in, out, dagger, -1);
}

// Mobius domain-wall operator D (dagger=0) or D^dag (dagger=1), full lattice.
void or_dwf(const Action* a, const cd* U, const cd* in, cd* out, int dagger) {
  dwf_full(*a, U, in, out, dagger);
}

// D or D^dag evaluated at n chosen 5D sites idx[k] = s*V + lex; out is n x 12.
// Used to check large lattices where the full oracle would take too long.
void or_dwf_sites(const Action* ap, const cd* U, const cd* in, const int64_t* idx, int64_t n,
                  cd* out, int dagger) {
  const Action& a = *ap;
  const long V = volume(a);
#pragma omp parallel for schedule(dynamic, 16)
  for (long k = 0; k < (long)n; ++k) {
    const int s = (int)(idx[k] / V);
    const long lex = idx[k] % V;
    cd* dst = out + k * 12;
    cd t[12], w[12];
    if (!dagger) {
      // chi = A in, formed on the fly wherever the hop reads it.
      auto chi = [&](int ss, long l, cd* r) {
        cd ct[12];
        cop_site(a, in, ss, l, 0, ct);
        const cd* src = spin_at(in, V, ss, l);
        for (int q = 0; q < 12; ++q) r[q] = a.b * src[q] + a.c * ct[q];
      };
      hop_site_fn(a, U, chi, s, lex, 0, w);
      cd c[12];
      chi(s, lex, c);
      cop_site(a, in, s, lex, 0, t);
      const cd* src = spin_at(in, V, s, lex);
      for (int q = 0; q < 12; ++q) dst[q] = (4.0 - a.M5) * c[q] - 0.5 * w[q] + src[q] - t[q];
    } else {
      // w_s' = D_W^dag in at (x, s') for s' in {s-1, s, s+1}; then A^dag w + B^dag in.
      cd wm[12], w0[12], wp[12];
      const int sm = (s - 1 + a.Ls) % a.Ls, sp = (s + 1) % a.Ls;
      auto dw = [&](int ss, cd* r) {
        hop_site(a, U, in, ss, lex, 1, r);
        const cd* src = spin_at(in, V, ss, lex);
        for (int q = 0; q < 12; ++q) r[q] = (4.0 - a.M5) * src[q] - 0.5 * r[q];
      };
      dw(sm, wm);
      dw(s, w0);
      dw(sp, wp);
      // C^dag w at s = P- (S_d w)_s + P+ (S_u w)_s
      const Gammas& G = gam();
      cd up[12], dn[12], cw[12];
      const double fu = (s + 1 < a.Ls) ? 1.0 : -a.mf;
      const double fd = (s - 1 >= 0) ? 1.0 : -a.mf;
      for (int q = 0; q < 12; ++q) { up[q] = fu * wp[q]; dn[q] = fd * wm[q]; cw[q] = 0; }
      spin_mat_acc(G.Pm, 1.0, dn, cw);
      spin_mat_acc(G.Pp, 1.0, up, cw);
      cop_site(a, in, s, lex, 1, t);
      const cd* src = spin_at(in, V, s, lex);
      for (int q = 0; q < 12; ++q) dst[q] = a.b * w0[q] + a.c * cw[q] + src[q] - t[q];
    }
  }
}

// x0 * f + x1 * C f (dagger=0) or with C^dag (dagger=1), every 5D site.
void or_local(const Action* a, const cd* in, cd* out, double x0, double x1, int dagger) {
  local_op(*a, in, out, x0, x1, dagger);
}

// M_ee (inverse=0) or M_ee^-1 (inverse=1), optionally adjoint, on every 4D site.
void or_mee(const Action* a, const cd* in, cd* out, int dagger, int inverse) {
  if (inverse) mee_inverse(*a, in, out, dagger);
  else local_op(*a, in, out, alpha_of(*a), beta_of(*a), dagger);
}

// Off-diagonal block with output parity p (input parity 1-p); see deo().
void or_deo(const Action* a, const cd* U, const cd* in, cd* out, int out_parity, int dagger) {
  deo(*a, U, in, out, out_parity, dagger);
}

// Schur complement M_pc (or M_pc^dag) on odd sites.
void or_mpc(const Action* a, const cd* U, const cd* in, cd* out, int dagger) {
  mpc(*a, U, in, out, dagger);
}

// CG on M_pc^dag M_pc x = b (odd sites), x0 = 0. Returns the iteration count;
// *true_res receives |b - A x| / |b| recomputed at exit.
int or_cg(const Action* ap, const cd* U, const cd* b, cd* x, double tol, int max_iter,
          double* true_res) {
  const Action& a = *ap;
  const size_t n = field_len(a);
  std::vector<cd> r(b, b + n), p(n), Ap(n), t(n);
  mask_parity(a, r.data(), 1);
  for (size_t k = 0; k < n; ++k) x[k] = 0;
  p = r;
  const double bb = dot_re(r.data(), r.data(), n);
  double rr = bb;
  int it = 0;
  while (it < max_iter && rr > tol * tol * bb) {
    mpc(a, U, p.data(), t.data(), 0);
    mpc(a, U, t.data(), Ap.data(), 1);
    const double pAp = dot_re(p.data(), Ap.data(), n);
    const double alpha = rr / pAp;
    for (size_t k = 0; k < n; ++k) {
      x[k] += alpha * p[k];
      r[k] -= alpha * Ap[k];
    }
    const double rr_new = dot_re(r.data(), r.data(), n);
    const double beta = rr_new / rr;
    rr = rr_new;
    for (size_t k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
    ++it;
  }
  mpc(a, U, x, t.data(), 0);
  mpc(a, U, t.data(), Ap.data(), 1);
  std::vector<cd> bo(b, b + n);
  mask_parity(a, bo.data(), 1);
  double res = 0;
  for (size_t k = 0; k < n; ++k) res += std::norm(bo[k] - Ap[k]);
  *true_res = std::sqrt(res / bb);
  return it;
}

}  // extern "C"
