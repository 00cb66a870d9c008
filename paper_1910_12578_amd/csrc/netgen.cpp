// Network code generator (see netgen.hpp).
//
// Reaction model (synthetic Arrhenius network, x = (rho X_1..rho X_Ns, rho e)):
//   k_r = exp(lnA_r + b_r ln T - E_r / T),  T = (gamma - 1) x_e / rho
//   v_r = k_r x_a            (unimolecular)   or  k_r x_a x_c  (bimolecular)
//   R_i = sum_r s_ir v_r,    R_e = sum_r Q_r v_r,  Q_r = -sum_i s_ir q_i.
// The Newton matrix is M = I - dt_m dR/dx.  Its LU factors are computed in a
// fixed order: for this class of networks every column of the species block
// of M sums to one, which keeps the diagonal at least half of the column's
// largest entry, so partial pivoting would not swap.  A run-time guard checks
// the ratio anyway and the kernel falls back to a pivoted dense solve when it
// fails.
#include "netgen.hpp"

#include <cmath>
#include <algorithm>
#include <cstdio>
#include <sstream>

namespace sdcgen {

static std::string num(double v) {
  char buf[64];
  std::snprintf(buf, sizeof buf, "%.17g", v);
  std::string s(buf);
  if (s.find_first_of(".eEn") == std::string::npos) s += ".0";
  return s;
}

Pattern build_pattern(const Topology& t) {
  Pattern p;
  const int n = t.ns + 1, e = t.ns;
  p.n = n;
  std::vector<char> S(n * n, 0);
  for (int i = 0; i < n; ++i) S[i * n + i] = 1;
  for (int r = 0; r < t.nr; ++r) {
    std::vector<int> cols;
    for (int a : t.reactants[r])
      if (a >= 0) cols.push_back(a);
    cols.push_back(e);
    for (int i = 0; i < t.ns; ++i)
      if (t.stoich[r * t.ns + i] != 0.0)
        for (int j : cols) S[i * n + j] = 1;
    for (int j : cols) S[e * n + j] = 1;  // energy row: Q_r dv_r/dx
  }
  int nj = 0;
  for (char c : S) nj += c;
  p.nnz_jac = nj;
  for (int k = 0; k < n; ++k)
    for (int i = k + 1; i < n; ++i)
      if (S[i * n + k])
        for (int j = k + 1; j < n; ++j)
          if (S[k * n + j]) {
            S[i * n + j] = 1;
            ++p.lu_fma;
          }
  p.index.assign(n * n, -1);
  int slot = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (S[i * n + j]) p.index[i * n + j] = slot++;
  p.nnz = slot;
  return p;
}

namespace {

struct Emit {
  std::ostringstream o;
  template <class T>
  Emit& operator<<(const T& v) {
    o << v;
    return *this;
  }
};

// Per-reaction quantities shared by the emitters.
struct Rx {
  int a, c;                     // reactants
  std::vector<std::pair<int, double>> s;  // (species, stoich) nonzeros
};

std::vector<Rx> reactions(const Topology& t) {
  std::vector<Rx> out(t.nr);
  for (int r = 0; r < t.nr; ++r) {
    out[r].a = t.reactants[r][0];
    out[r].c = t.reactants[r][1];
    for (int i = 0; i < t.ns; ++i) {
      double s = t.stoich[r * t.ns + i];
      if (s != 0.0) out[r].s.push_back({i, s});
    }
  }
  return out;
}

// "acc += s * val" with literal s, written without a multiply for +-1.
std::string accum(const std::string& acc, double s, const std::string& val) {
  if (s == 1.0) return acc + " += " + val + ";";
  if (s == -1.0) return acc + " -= " + val + ";";
  return acc + " = fma(" + num(s) + ", " + val + ", " + acc + ");";
}

std::string accum_t(const std::string& acc, double s, const std::string& val) {
  // matrix accumulation in the matrix type MT; val is already of type MT
  if (s == 1.0) return acc + " += " + val + ";";
  if (s == -1.0) return acc + " -= " + val + ";";
  return acc + " = fma((MT)" + num(s) + ", " + val + ", " + acc + ");";
}

void emit_rate(Emit& E, int r, const Rx& x) {
  E << "    const double k" << r << " = exp(fma(P->b[" << r << "], lnT, P->lnA[" << r
    << "]) - P->E[" << r << "] * invT);\n";
  if (x.c < 0)
    E << "    const double v" << r << " = k" << r << " * x[" << x.a << "];\n";
  else
    E << "    const double v" << r << " = k" << r << " * x[" << x.a << "] * x[" << x.c << "];\n";
}

// d v_r / d x_j for the reactant columns (as expressions) and the energy column.
std::vector<std::pair<int, std::string>> rate_derivs(int r, const Rx& x, int e) {
  std::vector<std::pair<int, std::string>> d;
  std::string k = "k" + std::to_string(r);
  if (x.c < 0) {
    d.push_back({x.a, k});
  } else if (x.a == x.c) {
    d.push_back({x.a, "2.0 * " + k + " * x[" + std::to_string(x.a) + "]"});
  } else {
    d.push_back({x.a, k + " * x[" + std::to_string(x.c) + "]"});
    d.push_back({x.c, k + " * x[" + std::to_string(x.a) + "]"});
  }
  d.push_back({e, "v" + std::to_string(r) + " * fma(P->E[" + std::to_string(r) +
                      "], invT2, P->b[" + std::to_string(r) + "] * invT) * dTdxe"});
  return d;
}

}  // namespace

FlopCount count_flops(const Topology& t, const Pattern& p) {
  FlopCount f;
  const int n = p.n;
  const auto rx = reactions(t);
  auto sacc = [](double s) { return (s == 1.0 || s == -1.0) ? 1 : 2; };
  // shared prologue: T = gm1 * x_e * irho (2), log (1), 1/T (1)
  f.source = 4;
  f.residual_matrix = 4 + 2 + n;  // + invT^2, dT/dx_e, G = x - b
  for (const auto& r : rx) {
    const long rate = 4 + 1 + (r.c < 0 ? 1 : 2);  // exp argument, exp, v
    f.source += rate + 2;                          // energy row fma
    for (auto& sp : r.s) f.source += sacc(sp.second);
    f.residual_matrix += rate + 1 + 2;             // g = -dt v, energy fma
    for (auto& sp : r.s) f.residual_matrix += 1 + sacc(sp.second);  // v*dtm and accumulate
    const int ncol = (r.c < 0 ? 1 : 2) + 1;
    f.residual_matrix += (r.c < 0 ? 0 : 2) + 5;    // reactant derivatives, energy derivative
    f.residual_matrix += ncol * (1 + 2);           // m_q = -dt * d, energy row
    for (auto& sp : r.s) f.residual_matrix += ncol * (sp.second == 1.0 || sp.second == -1.0 ? 1 : 2);
  }
  f.exps = t.nr;
  for (int k = 0; k < n; ++k) {
    int rows = 0, cols = 0;
    for (int i = k + 1; i < n; ++i) rows += p.index[i * n + k] >= 0;
    for (int j = k + 1; j < n; ++j) cols += p.index[k * n + j] >= 0;
    f.lu += 1 + rows + 2L * rows * cols;  // reciprocal, multipliers, updates
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (i != j && p.index[i * n + j] >= 0) f.solve += 2;
  f.solve += n;
  return f;
}

std::string generate(const Topology& t, const Pattern& p) {
  const int n = p.n, e = t.ns;
  const auto rx = reactions(t);
  Emit E;
  E << "// ---- generated network code: " << t.ns << " species, " << t.nr << " reactions\n";
  E << "// Newton matrix: " << p.nnz_jac << " structural nonzeros, " << p.nnz
    << " with LU fill-in, " << p.lu_fma << " factorisation multiply-adds\n";
  E << "#define SDC_NS " << t.ns << "\n#define SDC_NR " << t.nr << "\n#define SDC_NRA " << (t.nr > 0 ? t.nr : 1)
    << "\n#define SDC_NX " << n << "\n#define SDC_NNZ " << p.nnz << "\n\n";
  E << "struct NetParams { double lnA[SDC_NRA]; double b[SDC_NRA]; double E[SDC_NRA]; double Q[SDC_NRA]; "
       "double q[SDC_NS]; };\n";
  E << "// Rate parameters are staged once per block in LDS and read from there:\n"
       "// wave-uniform (broadcast) LDS reads, so the unrolled Newton loop keeps no\n"
       "// copy of them in scalar registers (which would spill into vector lanes).\n";
  E << "typedef const __attribute__((address_space(3))) NetParams* ParamPtr;\n\n";
  E << "// Reciprocal from the hardware estimate: two Newton steps in double (within\n"
       "// an ulp of 1/d, about half the cost of an IEEE division); the float\n"
       "// estimate alone is within an ulp.\n";
  E << "__device__ __forceinline__ double net_rcp(double d) {\n"
       "  double r = __builtin_amdgcn_rcp(d);\n"
       "  double e = fma(-d, r, 1.0);\n  r = fma(r, e, r);\n"
       "  e = fma(-d, r, 1.0);\n  return fma(r, e, r);\n}\n";
  E << "__device__ __forceinline__ float net_rcp(float d) { return __builtin_amdgcn_rcpf(d); }\n\n";

  // common prologue: temperature and its functions
  const char* prologue =
      "  const double T = gm1 * x[SDC_NX - 1] * irho;\n"
      "  const double lnT = log(T);\n"
      "  const double invT = 1.0 / T;\n";

  // ---- R(x)
  E << "// R(x; rho) on the reacting variables.\n";
  E << "__device__ __forceinline__ void net_source(const double* x, double irho, ParamPtr P, "
       "double gm1, double* R) {\n"
    << prologue;
  E << "  for (int i = 0; i < SDC_NX; ++i) R[i] = 0.0;\n";
  for (int r = 0; r < t.nr; ++r) {
    E << "  {\n";
    emit_rate(E, r, rx[r]);
    for (auto& [i, s] : rx[r].s) E << "    " << accum("R[" + std::to_string(i) + "]", s, "v" + std::to_string(r)) << "\n";
    E << "    R[" << e << "] = fma(P->Q[" << r << "], v" << r << ", R[" << e << "]);\n";
    E << "  }\n";
  }
  E << "}\n\n";

  // ---- residual G = x - b - dtm R and packed Newton matrix M = I - dtm dR/dx
  auto emit_residual_matrix = [&](bool dense) {
    if (!dense) {
      E << "// G = x - b - dt_m R(x) and the packed Newton matrix M = I - dt_m dR/dx.\n";
      E << "// XV: any type with double operator[](int) (a register array, or the\n"
           "// zone's slots of an LDS array that are read where they are needed).\n";
      E << "template <class MT, class XV>\n__device__ __forceinline__ void net_residual_matrix(const XV& x, const XV& b, "
           "double irho, double dtm, ParamPtr P, double gm1, double* G, MT* M) {\n";
    } else {
      E << "// Same as net_residual_matrix, into a dense row-major n x n array (pivoting fallback).\n";
      E << "__device__ __forceinline__ void net_residual_dense(const double* x, const double* b, double irho, "
           "double dtm, ParamPtr P, double gm1, double* G, double* M) {\n";
      E << "  typedef double MT;\n";
    }
    E << prologue;
    E << "  const double invT2 = invT * invT;\n  const double dTdxe = gm1 * irho;\n";
    E << "  for (int i = 0; i < SDC_NX; ++i) G[i] = x[i] - b[i];\n";
    if (dense) {
      E << "  for (int i = 0; i < SDC_NX * SDC_NX; ++i) M[i] = 0.0;\n";
      for (int i = 0; i < n; ++i) E << "  M[" << i * n + i << "] = 1.0;\n";
    } else {
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          int s = p.index[i * n + j];
          if (s >= 0) E << "  M[" << s << "] = (MT)" << (i == j ? "1" : "0") << ";\n";
        }
    }
    E << "  const double mdt = -dtm;\n";
    for (int r = 0; r < t.nr; ++r) {
      E << "  {\n";
      emit_rate(E, r, rx[r]);
      E << "    const double g" << r << " = mdt * v" << r << ";\n";
      for (auto& [i, s] : rx[r].s) E << "    " << accum("G[" + std::to_string(i) + "]", -s, "v" + std::to_string(r) + " * dtm") << "\n";
      E << "    G[" << e << "] = fma(P->Q[" << r << "], g" << r << ", G[" << e << "]);\n";
      auto d = rate_derivs(r, rx[r], e);
      for (size_t q = 0; q < d.size(); ++q) {
        int j = d[q].first;
        // one rounding to MT per derivative; the scatter runs in MT
        E << "    const MT m" << q << " = (MT)(mdt * (" << d[q].second << "));\n";
        for (auto& [i, s] : rx[r].s) {
          std::string slot = dense ? std::to_string(i * n + j) : std::to_string(p.index[i * n + j]);
          E << "    " << accum_t("M[" + slot + "]", s, "m" + std::to_string(q)) << "\n";
        }
        std::string slot = dense ? std::to_string(e * n + j) : std::to_string(p.index[e * n + j]);
        E << "    M[" << slot << "] = fma((MT)P->Q[" << r << "], m" << q << ", M[" << slot << "]);\n";
      }
      E << "  }\n";
    }
    E << "}\n\n";
  };
  emit_residual_matrix(false);

  // ---- topology tables for the compact, loop-based dense fallback
  {
    size_t maxs = 1;
    for (auto& r : rx) maxs = std::max(maxs, r.s.size());
    const int nra = t.nr > 0 ? t.nr : 1;
    E << "// Topology tables (dense pivoting fallback): reactants, species and stoichiometry.\n";
    E << "#define SDC_MAXS " << maxs << "\n";
    auto emit_int = [&](const char* name, auto get) {
      E << "__constant__ int " << name << "[" << nra << "] = {";
      for (int r = 0; r < nra; ++r) E << (r ? ", " : "") << (r < t.nr ? get(r) : 0);
      E << "};\n";
    };
    emit_int("kRxA", [&](int r) { return rx[r].a; });
    emit_int("kRxC", [&](int r) { return rx[r].c; });
    emit_int("kRxN", [&](int r) { return (int)rx[r].s.size(); });
    E << "__constant__ int kRxSp[" << nra << "][SDC_MAXS] = {";
    for (int r = 0; r < nra; ++r) {
      E << (r ? ", " : "") << "{";
      for (size_t q = 0; q < maxs; ++q) E << (q ? ", " : "") << (r < t.nr && q < rx[r].s.size() ? rx[r].s[q].first : 0);
      E << "}";
    }
    E << "};\n__constant__ double kRxS[" << nra << "][SDC_MAXS] = {";
    for (int r = 0; r < nra; ++r) {
      E << (r ? ", " : "") << "{";
      for (size_t q = 0; q < maxs; ++q) E << (q ? ", " : "") << (r < t.nr && q < rx[r].s.size() ? num(rx[r].s[q].second) : "0.0");
      E << "}";
    }
    E << "};\n\n";
  }

  // ---- LU in place, diagonal slots receive 1/pivot; returns false if a
  // pivot is smaller than tau times the largest entry of its column.
  E << "// In-place LU of the packed matrix in the fixed order; diagonal slots hold 1/pivot.\n";
  E << "template <class MT>\n__device__ __forceinline__ bool net_lu(MT* M, MT tau) {\n  bool ok = true;\n";
  for (int k = 0; k < n; ++k) {
    int dk = p.index[k * n + k];
    std::vector<int> rows, cols;
    for (int i = k + 1; i < n; ++i)
      if (p.index[i * n + k] >= 0) rows.push_back(i);
    for (int j = k + 1; j < n; ++j)
      if (p.index[k * n + j] >= 0) cols.push_back(j);
    E << "  {\n    const MT piv = M[" << dk << "];\n";
    if (!rows.empty()) {
      E << "    MT cmax = fabs(piv);\n";
      for (int i : rows) E << "    cmax = fmax(cmax, fabs(M[" << p.index[i * n + k] << "]));\n";
      E << "    ok = ok && (fabs(piv) >= tau * cmax);\n";
    } else {
      E << "    ok = ok && (fabs(piv) >= tau * fabs(piv)) && (piv != (MT)0);\n";
    }
    E << "    const MT inv = net_rcp(piv);\n    M[" << dk << "] = inv;\n";
    for (int i : rows) {
      int li = p.index[i * n + k];
      E << "    { const MT l = M[" << li << "] * inv; M[" << li << "] = l;\n";
      for (int j : cols) E << "      M[" << p.index[i * n + j] << "] = fma(-l, M[" << p.index[k * n + j] << "], M[" << p.index[i * n + j] << "]);\n";
      E << "    }\n";
    }
    E << "  }\n";
  }
  E << "  return ok;\n}\n\n";

  // ---- LU with the forward substitution folded in: each multiplier updates
  // the right-hand side as soon as it is formed and is then dropped (only U
  // stays live), followed by the backward substitution.  The operations on r
  // are those of a forward substitution with the factors of net_lu (k
  // ascending) and a backward one, in the same order.
  E << "// Factor and solve in one pass: r <- M^{-1} r; M keeps U (diagonal 1/pivot), not L.\n";
  E << "template <class MT>\n__device__ __forceinline__ bool net_lu_solve(MT* M, MT* r, MT tau) {\n  bool ok = true;\n";
  for (int k = 0; k < n; ++k) {
    int dk = p.index[k * n + k];
    std::vector<int> rows, cols;
    for (int i = k + 1; i < n; ++i)
      if (p.index[i * n + k] >= 0) rows.push_back(i);
    for (int j = k + 1; j < n; ++j)
      if (p.index[k * n + j] >= 0) cols.push_back(j);
    E << "  {\n    const MT piv = M[" << dk << "];\n";
    if (!rows.empty()) {
      E << "    MT cmax = fabs(piv);\n";
      for (int i : rows) E << "    cmax = fmax(cmax, fabs(M[" << p.index[i * n + k] << "]));\n";
      E << "    ok = ok && (fabs(piv) >= tau * cmax);\n";
    } else {
      E << "    ok = ok && (fabs(piv) >= tau * fabs(piv)) && (piv != (MT)0);\n";
    }
    E << "    const MT inv = net_rcp(piv);\n    M[" << dk << "] = inv;\n";
    for (int i : rows) {
      int li = p.index[i * n + k];
      E << "    { const MT l = M[" << li << "] * inv;\n";
      E << "      r[" << i << "] = fma(-l, r[" << k << "], r[" << i << "]);\n";
      for (int j : cols) E << "      M[" << p.index[i * n + j] << "] = fma(-l, M[" << p.index[k * n + j] << "], M[" << p.index[i * n + j] << "]);\n";
      E << "    }\n";
    }
    E << "  }\n";
  }
  for (int k = n - 1; k >= 0; --k) {
    for (int j = k + 1; j < n; ++j)
      if (p.index[k * n + j] >= 0) E << "  r[" << k << "] = fma(-M[" << p.index[k * n + j] << "], r[" << j << "], r[" << k << "]);\n";
    E << "  r[" << k << "] *= M[" << p.index[k * n + k] << "];\n";
  }
  E << "  return ok;\n}\n\n";

  // ---- transpose solve: r <- (LU)^{-T} r  (adjoint of the implicit solve)
  E << "// Solve with the transposed factors: r <- (LU)^{-T} r.\n";
  E << "template <class MT>\n__device__ __forceinline__ void net_solve_t(const MT* M, MT* r) {\n";
  for (int k = 0; k < n; ++k) {
    for (int j = 0; j < k; ++j)
      if (p.index[j * n + k] >= 0) E << "  r[" << k << "] = fma(-M[" << p.index[j * n + k] << "], r[" << j << "], r[" << k << "]);\n";
    E << "  r[" << k << "] *= M[" << p.index[k * n + k] << "];\n";
  }
  for (int k = n - 1; k >= 0; --k)
    for (int i = k + 1; i < n; ++i)
      if (p.index[i * n + k] >= 0) E << "  r[" << k << "] = fma(-M[" << p.index[i * n + k] << "], r[" << i << "], r[" << k << "]);\n";
  E << "}\n\n";

  // ---- vector-Jacobian products of R for the adjoint:
  //   xbar += (dR/dx)^T w, and d(w.R)/d rho at fixed x, d(w.R)/d lnA_r, d(w.R)/dE_r.
  E << "// Adjoint helpers at fixed rho: xbar = (dR/dx)^T w, rhobar = d(w.R)/drho,\n"
       "// gl[r] += d(w.R)/dlnA_r, gE[r] += d(w.R)/dE_r (accumulated).\n";
  E << "__device__ __forceinline__ void net_vjp(const double* x, double irho, ParamPtr P, "
       "double gm1, const double* w, double* xbar, double* rhobar, double* gl, double* gE) {\n"
    << prologue;
  E << "  const double invT2 = invT * invT;\n  const double dTdxe = gm1 * irho;\n";
  E << "  for (int i = 0; i < SDC_NX; ++i) xbar[i] = 0.0;\n  double tbar = 0.0;\n";
  for (int r = 0; r < t.nr; ++r) {
    E << "  {\n";
    emit_rate(E, r, rx[r]);
    // wr = sum_i w_i s_ir + w_e Q_r  (sensitivity of w.R to v_r)
    E << "    double wr = P->Q[" << r << "] * w[" << e << "];\n";
    for (auto& [i, s] : rx[r].s) E << "    " << accum("wr", s, "w[" + std::to_string(i) + "]") << "\n";
    auto d = rate_derivs(r, rx[r], e);
    for (size_t q = 0; q + 1 < d.size(); ++q) E << "    xbar[" << d[q].first << "] = fma(wr, " << d[q].second << ", xbar[" << d[q].first << "]);\n";
    // dv/dT = v (b/T + E/T^2): enters through x_e (dT/dx_e) and rho (dT/drho = -T/rho)
    E << "    const double dvdT = v" << r << " * fma(P->E[" << r << "], invT2, P->b[" << r << "] * invT);\n";
    E << "    tbar = fma(wr, dvdT, tbar);\n";
    E << "    gl[" << r << "] = fma(wr, v" << r << ", gl[" << r << "]);\n";
    E << "    gE[" << r << "] = fma(-wr, v" << r << " * invT, gE[" << r << "]);\n";
    E << "  }\n";
  }
  E << "  xbar[" << e << "] = fma(tbar, dTdxe, xbar[" << e << "]);\n";
  E << "  *rhobar = -tbar * T * irho;\n";
  E << "}\n";
  return E.o.str();
}

}  // namespace sdcgen
