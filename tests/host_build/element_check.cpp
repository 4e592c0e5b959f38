// Host build of the library's per-lane algebra for checks under
// AddressSanitizer and UndefinedBehaviorSanitizer.
//
// For seeded random operands it evaluates, in both element forms (matrices,
// operators.hpp; lower-triangular factors, sqrt.hpp), the filtering element
// (eq. 13-14), the filtering operator and its carry application (eq. 15), the
// smoothing element (eq. 17-18) and the smoothing operator (eq. 19), and
// prints one JSON object per case with the inputs and both results (factors
// multiplied out).  tests/test_host_build.py compares them with the oracle.
//
//   element_check <seed> <cases>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>

#include "elements.hpp"
#include "operators.hpp"
#include "sqrt.hpp"

using namespace pks;

namespace {

std::mt19937_64 rng;

double unif(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

template <int M, int K>
void rand_mat(double (&A)[M][K], double s) {
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < K; ++j) A[i][j] = unif(-s, s);
}
template <int M>
void rand_vec(double (&a)[M], double s) {
  for (int i = 0; i < M; ++i) a[i] = unif(-s, s);
}
// random lower-triangular factor with a positive diagonal
template <int N>
void rand_tril(double (&L)[N][N], double s) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) L[i][j] = j < i ? unif(-s, s) : (j == i ? unif(0.3, 1.5) * s : 0.0);
}
// A = L L^T
template <int N, int K>
void gram_of(const double (&L)[N][K], double (&A)[N][N]) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double t = 0.0;
      for (int k = 0; k < K; ++k) t += L[i][k] * L[j][k];
      A[i][j] = t;
    }
}

std::string out;
bool first_field = true;

void open_case(const char* kind, int n, int p) {
  out = std::string("{\"kind\": \"") + kind + "\", \"n\": " + std::to_string(n) + ", \"p\": " + std::to_string(p);
}
template <int M, int K, typename R>
void field(const char* name, const R (&A)[M][K]) {
  out += std::string(", \"") + name + "\": [";
  char buf[40];
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < K; ++j) {
      std::snprintf(buf, sizeof buf, "%s%.17g", (i || j) ? ", " : "", double(A[i][j]));
      out += buf;
    }
  out += "]";
}
template <int M, typename R>
void field(const char* name, const R (&a)[M]) {
  out += std::string(", \"") + name + "\": [";
  char buf[40];
  for (int i = 0; i < M; ++i) {
    std::snprintf(buf, sizeof buf, "%s%.17g", i ? ", " : "", double(a[i]));
    out += buf;
  }
  out += "]";
}
void close_case() { std::printf("%s}\n", out.c_str()); }

template <int N, typename R>
void to_r(const double (&A)[N][N], R (&B)[N][N]) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) B[i][j] = R(A[i][j]);
}
template <int N, typename R>
void to_r(const double (&a)[N], R (&b)[N]) {
  for (int i = 0; i < N; ++i) b[i] = R(a[i]);
}
template <int N, typename R>
void gram_r(const R (&L)[N][N], R (&A)[N][N]) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      R t = R(0);
      for (int k = 0; k < N; ++k) t += L[i][k] * L[j][k];
      A[i][j] = t;
    }
}

// A random filtering element in both forms: C = U U^T, J = Z Z^T (rank p).
template <int N, int P, typename R>
void rand_filter_elem(FilterElem<N, R>& c, SqrtFilterElem<N, R>& s, double (&Cd)[N][N], double (&Jd)[N][N],
                      double (&Ad)[N][N], double (&bd)[N], double (&etad)[N]) {
  double U[N][N], Y[N][P], Z[N][N] = {};
  rand_tril<N>(U, 1.0);
  rand_mat<N, P>(Y, 1.0);
  rand_mat<N, N>(Ad, 1.0);
  rand_vec<N>(bd, 2.0);
  rand_vec<N>(etad, 2.0);
  gram_of<N, N>(U, Cd);
  gram_of<N, P>(Y, Jd);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < P; ++j) Z[i][j] = Y[i][j];
  to_r(Ad, c.A);
  to_r(bd, c.b);
  to_r(Cd, c.C);
  to_r(etad, c.eta);
  to_r(Jd, c.J);
  to_r(Ad, s.A);
  to_r(bd, s.b);
  to_r(U, s.U);
  to_r(etad, s.eta);
  // the stored factor is triangular: tria of [Y, 0]
  R Zr[N][N];
  to_r(Z, Zr);
  tria<N, N>(Zr, s.Z);
}

template <int N, int P, typename R>
void filter_cases(int count, const char* tag) {
  for (int k = 0; k < count; ++k) {
    // ---- element from a random surrogate model
    {
      double F[N][N], c[N], Uq[N][N], Qp[N][N], H[P][N], d[P], Ur[P][P], Rp[P][P], y[P];
      rand_mat<N, N>(F, 1.0);
      rand_vec<N>(c, 1.0);
      rand_tril<N>(Uq, 0.5);
      gram_of<N, N>(Uq, Qp);
      rand_mat<P, N>(H, 1.0);
      rand_vec<P>(d, 1.0);
      rand_tril<P>(Ur, 0.5);
      gram_of<P, P>(Ur, Rp);
      rand_vec<P>(y, 2.0);
      R Fr[N][N], cr[N], Qr[N][N], Hr[P][N], dr[P], Rr[P][P], yr[P];
      to_r(F, Fr);
      to_r(c, cr);
      to_r(Qp, Qr);
      for (int i = 0; i < P; ++i)
        for (int j = 0; j < N; ++j) Hr[i][j] = R(H[i][j]);
      to_r(d, dr);
      to_r(Rp, Rr);
      to_r(y, yr);
      FilterElem<N, R> e;
      SqrtFilterElem<N, R> q;
      const bool ok1 = filter_element<N, P, R>(Fr, cr, Qr, Hr, dr, Rr, yr, e.A, e.b, e.C, e.eta, e.J);
      const bool ok2 = sqrt_filter_element<N, P, R>(Fr, cr, Qr, Hr, dr, Rr, yr, q.A, q.b, q.U, q.eta, q.Z);
      R qC[N][N], qJ[N][N];
      gram_r<N>(q.U, qC);
      gram_r<N>(q.Z, qJ);
      open_case("filter_element", N, P);
      out += std::string(", \"prec\": \"") + tag + "\", \"ok\": " + ((ok1 && ok2) ? "true" : "false");
      field("F", F), field("c", c), field("Qp", Qp), field("H", H), field("d", d), field("Rp", Rp), field("y", y);
      field("cov_A", e.A), field("cov_b", e.b), field("cov_C", e.C), field("cov_eta", e.eta), field("cov_J", e.J);
      field("sq_A", q.A), field("sq_b", q.b), field("sq_C", qC), field("sq_eta", q.eta), field("sq_J", qJ);
      field("sq_U", q.U), field("sq_Z", q.Z);
      close_case();
    }
    // ---- combine of two random elements, and a carry applied to one
    {
      FilterElem<N, R> ci, cj, co;
      SqrtFilterElem<N, R> si, sj, so;
      double Ci[N][N], Ji[N][N], Ai[N][N], bi[N], ei[N], Cj[N][N], Jj[N][N], Aj[N][N], bj[N], ej[N];
      rand_filter_elem<N, P, R>(ci, si, Ci, Ji, Ai, bi, ei);
      rand_filter_elem<N, P, R>(cj, sj, Cj, Jj, Aj, bj, ej);
      FilterOp<N, R, true>::combine(ci, cj, co);
      SqrtFilterOp<N, R, true>::combine(si, sj, so);
      R sC[N][N], sJ[N][N];
      gram_r<N>(so.U, sC);
      gram_r<N>(so.Z, sJ);
      open_case("filter_combine", N, P);
      out += std::string(", \"prec\": \"") + tag + "\"";
      field("Ai", Ai), field("bi", bi), field("Ci", Ci), field("etai", ei), field("Ji", Ji);
      field("Aj", Aj), field("bj", bj), field("Cj", Cj), field("etaj", ej), field("Jj", Jj);
      field("cov_A", co.A), field("cov_b", co.b), field("cov_C", co.C), field("cov_eta", co.eta), field("cov_J", co.J);
      field("sq_A", so.A), field("sq_b", so.b), field("sq_C", sC), field("sq_eta", so.eta), field("sq_J", sJ);
      field("sq_U", so.U), field("sq_Z", so.Z);
      close_case();
      // carry (b_i, C_i) applied to a_j: the combine with A_i = 0, eta_i = J_i = 0
      FilterCarry<N, R> cc, cco;
      SqrtFilterCarry<N, R> sc, sco;
      for (int i = 0; i < N; ++i) {
        cc.b[i] = ci.b[i];
        sc.b[i] = si.b[i];
        for (int j = 0; j < N; ++j) {
          cc.C[i][j] = ci.C[i][j];
          sc.U[i][j] = si.U[i][j];
        }
      }
      FilterOp<N, R, true>::apply(cc, cj, cco);
      SqrtFilterOp<N, R, true>::apply(sc, sj, sco);
      R aC[N][N];
      gram_r<N>(sco.U, aC);
      open_case("filter_apply", N, P);
      out += std::string(", \"prec\": \"") + tag + "\"";
      field("bi", bi), field("Ci", Ci);
      field("Aj", Aj), field("bj", bj), field("Cj", Cj), field("etaj", ej), field("Jj", Jj);
      field("cov_b", cco.b), field("cov_C", cco.C), field("sq_b", sco.b), field("sq_C", aC);
      close_case();
    }
  }
}

template <int N, typename R>
void smoother_cases(int count, const char* tag) {
  for (int k = 0; k < count; ++k) {
    {
      double x[N], U[N][N], P[N][N], F[N][N], c[N], Uq[N][N], Qp[N][N];
      rand_vec<N>(x, 2.0);
      rand_tril<N>(U, 1.0);
      gram_of<N, N>(U, P);
      rand_mat<N, N>(F, 1.0);
      rand_vec<N>(c, 1.0);
      rand_tril<N>(Uq, 0.5);
      gram_of<N, N>(Uq, Qp);
      R xr[N], Pr[N][N], Ur[N][N], Fr[N][N], cr[N], Qr[N][N];
      to_r(x, xr);
      to_r(P, Pr);
      to_r(U, Ur);
      to_r(F, Fr);
      to_r(c, cr);
      to_r(Qp, Qr);
      SmootherElem<N, R> e;
      SqrtSmootherElem<N, R> q;
      const bool ok1 = smoother_element<N, R>(xr, Pr, Fr, cr, Qr, e.E, e.g, e.L);
      const bool ok2 = sqrt_smoother_element<N, R>(xr, Ur, Fr, cr, Qr, q.E, q.g, q.D);
      R qL[N][N];
      gram_r<N>(q.D, qL);
      open_case("smoother_element", N, 0);
      out += std::string(", \"prec\": \"") + tag + "\", \"ok\": " + ((ok1 && ok2) ? "true" : "false");
      field("x", x), field("P", P), field("F", F), field("c", c), field("Qp", Qp);
      field("cov_E", e.E), field("cov_g", e.g), field("cov_L", e.L);
      field("sq_E", q.E), field("sq_g", q.g), field("sq_L", qL), field("sq_D", q.D);
      close_case();
    }
    {
      // y (x) x in scan order = paper's a_i (x) a_j with a_i = y (earlier slot), a_j = x
      double Ei[N][N], gi[N], Di[N][N], Li[N][N], Ej[N][N], gj[N], Dj[N][N], Lj[N][N];
      rand_mat<N, N>(Ei, 0.8);
      rand_vec<N>(gi, 2.0);
      rand_tril<N>(Di, 1.0);
      gram_of<N, N>(Di, Li);
      rand_mat<N, N>(Ej, 0.8);
      rand_vec<N>(gj, 2.0);
      rand_tril<N>(Dj, 1.0);
      gram_of<N, N>(Dj, Lj);
      SmootherElem<N, R> ci, cj, co;
      SqrtSmootherElem<N, R> si, sj, so;
      to_r(Ei, ci.E), to_r(gi, ci.g), to_r(Li, ci.L), to_r(Ej, cj.E), to_r(gj, cj.g), to_r(Lj, cj.L);
      to_r(Ei, si.E), to_r(gi, si.g), to_r(Di, si.D), to_r(Ej, sj.E), to_r(gj, sj.g), to_r(Dj, sj.D);
      SmootherOp<N, R, true>::combine(cj, ci, co);
      SqrtSmootherOp<N, R, true>::combine(sj, si, so);
      R sL[N][N];
      gram_r<N>(so.D, sL);
      open_case("smoother_combine", N, 0);
      out += std::string(", \"prec\": \"") + tag + "\"";
      field("Ei", Ei), field("gi", gi), field("Li", Li), field("Ej", Ej), field("gj", gj), field("Lj", Lj);
      field("cov_E", co.E), field("cov_g", co.g), field("cov_L", co.L);
      field("sq_E", so.E), field("sq_g", so.g), field("sq_L", sL);
      close_case();
    }
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: element_check <seed> <cases>\n");
    return 2;
  }
  rng.seed(std::strtoull(argv[1], nullptr, 10));
  const int count = std::atoi(argv[2]);
  filter_cases<5, 2, double>(count, "f64");
  filter_cases<3, 2, double>(count, "f64");
  filter_cases<1, 1, double>(count, "f64");
  filter_cases<5, 2, float>(count, "f32");
  smoother_cases<5, double>(count, "f64");
  smoother_cases<3, double>(count, "f64");
  smoother_cases<5, float>(count, "f32");
  return 0;
}
