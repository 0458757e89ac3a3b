// Host generation of every dense matrix the box code applies (built once per process).
//
// Near tables (the volume quadrature of adjacent leaves, Sec. 4.2 eq. (vbulk) restricted to a
// pair of touching leaves) in target half-widths:
//     T_r[m,k] = -(1/2pi) [ ln(rho_r) W_k + I_k((xi_m - d_r)/rho_r) ],
//     I_k(x0)  = int_{[-1,1]^2} ln|y - x0| l_k(y) dy,
// computed here independently of any other code path:
//   * x0 inside the square (self relation): four triangles with apex x0 in Duffy coordinates
//     y = x0 + u (P0 - x0 + v (P1 - P0)); ln|y - x0| = ln u + ln|E(v)|. The u integral of
//     u (ln u + c) poly(u) (degree <= 31) is exact with 32 Gauss-Legendre nodes and
//     product-integration weights for ln u (Legendre moments int_0^1 ln(u) P*_n(u) du =
//     (-1)^(n+1)/(n(n+1))); the v integral uses Gauss panels refined until the complex
//     singularity of ln|E(v)| lies outside the Bernstein ellipse of parameter 4.
//   * x0 outside (all other relations): a tensor mesh graded geometrically towards the
//     nearest boundary point p, breakpoints p +- h 2^(k-1) (h = |x0 - p|), 24-point Gauss in
//     each direction, applied as Lx diag(w G) Ly^T.
// D4 symmetry: only the 7 relation classes are integrated; the other 26 tables are the same
// numbers with rows and columns permuted alike.
//
// Far-field matrices follow the Greengard-Rokhlin expansions in scaled form (multipole
// phi(z) = a_0 ln(z-c) + sum a_n (s/(z-c))^n, local psi(z) = sum b_l ((z-c)/s)^l, complex
// z = x + iy, G = -(1/2pi) Re ln z), converted to real matrices on interleaved (Re, Im).
#include <algorithm>
#include <atomic>
#include <stdexcept>
#include <cmath>
#include <complex>
#include <map>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <string>
#include <thread>

#include "plan.hpp"
#include "moments.hpp"

namespace vp {

using cd = std::complex<double>;
static const double kInv2Pi = 1.0 / (2.0 * M_PI);

// ---------------------------------------------------------------- 1D rules and basis
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

struct Basis {
  double t[kP], lam[kP], w[kP], W[kNP];
  Basis() {
    for (int i = 0; i < kP; ++i) t[i] = -std::cos((2.0 * i + 1.0) * M_PI / (2.0 * kP));
    for (int i = 0; i < kP; ++i) {
      double v = 1.0;
      for (int j = 0; j < kP; ++j)
        if (j != i) v *= (t[i] - t[j]);
      lam[i] = 1.0 / v;
    }
    // Fejer first-rule weights (interpolatory weights of these points)
    for (int i = 0; i < kP; ++i) {
      double th = std::acos(t[i]), s = 0.0;
      for (int j = 1; j <= kP / 2; ++j) s += std::cos(2.0 * j * th) / (4.0 * j * j - 1.0);
      w[i] = (2.0 / kP) * (1.0 - 2.0 * s);
    }
    for (int j = 0; j < kP; ++j)
      for (int i = 0; i < kP; ++i) W[j * kP + i] = w[i] * w[j];
  }
  void lagrange(double x, double* L) const {
    for (int i = 0; i < kP; ++i)
      if (x == t[i]) {
        for (int j = 0; j < kP; ++j) L[j] = (i == j) ? 1.0 : 0.0;
        return;
      }
    double s = 0.0;
    for (int i = 0; i < kP; ++i) {
      L[i] = lam[i] / (x - t[i]);
      s += L[i];
    }
    for (int i = 0; i < kP; ++i) L[i] /= s;
  }
};
static const Basis& basis() { static const Basis b; return b; }

// ---------------------------------------------------------------- near: x0 inside
struct LogRule {
  std::vector<double> u, w, wl;  // 32 GL nodes on [0,1], weights, ln-product weights
  LogRule() {
    std::vector<double> x, ww;
    gauss_legendre(32, x, ww);
    u.resize(32); w.resize(32); wl.resize(32);
    for (int j = 0; j < 32; ++j) { u[j] = 0.5 * (x[j] + 1.0); w[j] = 0.5 * ww[j]; }
    for (int j = 0; j < 32; ++j) {
      // shifted Legendre P*_n(u) = P_n(2u - 1)
      double z = 2.0 * u[j] - 1.0, p0 = 1.0, p1 = z, s = -1.0;  // n = 0 term: (2*0+1) P0 M0 = -1
      s += 3.0 * p1 * 0.5;  // n = 1: M1 = +1/2
      for (int n = 2; n < 32; ++n) {
        double p2 = ((2.0 * n - 1.0) * z * p1 - (n - 1.0) * p0) / n;
        p0 = p1;
        p1 = p2;
        double Mn = ((n + 1) % 2 == 0 ? 1.0 : -1.0) / (double(n) * (n + 1));
        s += (2.0 * n + 1.0) * p1 * Mn;
      }
      wl[j] = w[j] * s;
    }
  }
};

static double bernstein_rho(cd z, double c, double hl) {
  cd w = (z - c) / hl;
  cd s = std::sqrt(w - 1.0) * std::sqrt(w + 1.0);
  return std::max(std::abs(w + s), std::abs(w - s));
}

static void accumulate_point(const Basis& B, double y1, double y2, double wt, double* I) {
  double Lx[kP], Ly[kP];
  B.lagrange(y1, Lx);
  B.lagrange(y2, Ly);
  for (int j = 0; j < kP; ++j) {
    double a = wt * Ly[j];
    double* row = I + j * kP;
    for (int i = 0; i < kP; ++i) row[i] += a * Lx[i];
  }
}

static void inside_triangle(const Basis& B, const LogRule& R, const std::vector<double>& gx,
                            const std::vector<double>& gw, double x0, double y0, double p0x, double p0y,
                            double p1x, double p1y, double* I) {
  double e0x = p0x - x0, e0y = p0y - y0, dx = p1x - p0x, dy = p1y - p0y;
  double twoA = std::fabs(e0x * dy - e0y * dx);
  if (twoA < 1e-300) return;
  double L2 = dx * dx + dy * dy, L = std::sqrt(L2);
  double vf = -(e0x * dx + e0y * dy) / L2, hv = twoA / L / L;  // singularities at vf +- i hv
  cd zs(vf, hv);
  std::vector<std::pair<double, double>> stack{{0.0, 1.0}}, panels;
  while (!stack.empty()) {
    auto pr = stack.back();
    stack.pop_back();
    double c = 0.5 * (pr.first + pr.second), hl = 0.5 * (pr.second - pr.first);
    if (bernstein_rho(zs, c, hl) >= 4.0 || hl < 1e-12) panels.push_back(pr);
    else { stack.push_back({pr.first, c}); stack.push_back({c, pr.second}); }
  }
  for (auto& pr : panels) {
    double c = 0.5 * (pr.first + pr.second), hl = 0.5 * (pr.second - pr.first);
    for (size_t q = 0; q < gx.size(); ++q) {
      double v = c + hl * gx[q], wv = hl * gw[q];
      double ex = e0x + v * dx, ey = e0y + v * dy;
      double lnE = 0.5 * std::log(ex * ex + ey * ey);
      for (int j = 0; j < 32; ++j) {
        double u = R.u[j];
        double wt = twoA * wv * u * (R.wl[j] + lnE * R.w[j]);
        accumulate_point(B, x0 + u * ex, y0 + u * ey, wt, I);
      }
    }
  }
}

// ---------------------------------------------------------------- near: x0 outside
static std::vector<double> graded_breaks(double p, double h) {
  std::vector<double> b{-1.0, 1.0};
  for (double d = 0.5 * h; d < 2.0; d *= 2.0) {
    if (p - d > -1.0) b.push_back(p - d);
    if (p + d < 1.0) b.push_back(p + d);
  }
  std::sort(b.begin(), b.end());
  b.erase(std::unique(b.begin(), b.end(), [](double a, double c) { return std::fabs(a - c) < 1e-15; }), b.end());
  return b;
}

static void outside_graded(const Basis& B, double x0, double y0, double* I) {
  double px = std::min(1.0, std::max(-1.0, x0)), py = std::min(1.0, std::max(-1.0, y0));
  double h = std::hypot(x0 - px, y0 - py);
  std::vector<double> bx = graded_breaks(px, h), by = graded_breaks(py, h);
  static thread_local std::vector<double> gx, gw;
  if (gx.empty()) gauss_legendre(24, gx, gw);
  const int n = 24;
  double Lx[24][kP], Ly[24][kP], G[24][24], C[kP][24];
  for (size_t a = 0; a + 1 < bx.size(); ++a) {
    double cx = 0.5 * (bx[a] + bx[a + 1]), hx = 0.5 * (bx[a + 1] - bx[a]);
    for (int q = 0; q < n; ++q) B.lagrange(cx + hx * gx[q], Lx[q]);
    for (size_t b = 0; b + 1 < by.size(); ++b) {
      double cy = 0.5 * (by[b] + by[b + 1]), hy = 0.5 * (by[b + 1] - by[b]);
      for (int q = 0; q < n; ++q) B.lagrange(cy + hy * gx[q], Ly[q]);
      for (int qa = 0; qa < n; ++qa) {
        double ddx = cx + hx * gx[qa] - x0;
        for (int qb = 0; qb < n; ++qb) {
          double ddy = cy + hy * gx[qb] - y0;
          G[qa][qb] = 0.5 * std::log(ddx * ddx + ddy * ddy) * gw[qa] * gw[qb] * hx * hy;
        }
      }
      for (int i = 0; i < kP; ++i)
        for (int qb = 0; qb < n; ++qb) {
          double s = 0.0;
          for (int qa = 0; qa < n; ++qa) s += Lx[qa][i] * G[qa][qb];
          C[i][qb] = s;
        }
      for (int j = 0; j < kP; ++j)
        for (int i = 0; i < kP; ++i) {
          double s = 0.0;
          for (int qb = 0; qb < n; ++qb) s += C[i][qb] * Ly[qb][j];
          I[j * kP + i] += s;
        }
    }
  }
}

static void logint(double x0, double y0, double* I) {
  const Basis& B = basis();
  std::memset(I, 0, sizeof(double) * kNP);
  if (std::fabs(x0) < 1.0 && std::fabs(y0) < 1.0) {
    static const LogRule R;
    static thread_local std::vector<double> gx, gw;
    if (gx.empty()) gauss_legendre(32, gx, gw);
    const double P[5][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}, {-1, -1}};
    for (int e = 0; e < 4; ++e) inside_triangle(B, R, gx, gw, x0, y0, P[e][0], P[e][1], P[e + 1][0], P[e + 1][1], I);
  } else {
    outside_graded(B, x0, y0, I);
  }
}

// ---------------------------------------------------------------- moments at an arbitrary point
// For xi = (x0, y0) anywhere: I_k = int log|xi - eta| l_k(eta) d eta and (Ix_k, Iy_k) =
// int (xi - eta) / |xi - eta|^2 l_k(eta) d eta over the reference square (the gradient of I in
// xi). The square is refined towards xi as a quadtree: a square at distance >= its side from
// xi takes a 24 x 24 tensor Gauss rule (the kernels are analytic there); a square of
// half-width <= 1/32 whose closure holds xi takes four
// polar-Duffy triangles with apex xi (a 16-point log-product rule in the radial variable, exact
// to degree 15, which on so small a square leaves terms of relative size 32^-16; adaptive
// 12-point panels along the far edge, as for the tables). The gradient kernel times the Duffy
// Jacobian u is smooth in u and takes the plain Gauss weights.
struct LogRule16 {
  double u[16], w[16], wl[16];
  LogRule16() {
    std::vector<double> x, ww;
    gauss_legendre(16, x, ww);
    for (int j = 0; j < 16; ++j) { u[j] = 0.5 * (x[j] + 1.0); w[j] = 0.5 * ww[j]; }
    for (int j = 0; j < 16; ++j) {  // interpolatory weights of int_0^1 ln(u) p(u) du (shifted Legendre moments)
      double z = 2.0 * u[j] - 1.0, p0 = 1.0, p1 = z, sum = -1.0 + 3.0 * p1 * 0.5;
      for (int n = 2; n < 16; ++n) {
        double p2 = ((2.0 * n - 1.0) * z * p1 - (n - 1.0) * p0) / n;
        p0 = p1;
        p1 = p2;
        sum += (2.0 * n + 1.0) * p1 * (((n + 1) % 2 == 0 ? 1.0 : -1.0) / (double(n) * (n + 1)));
      }
      wl[j] = w[j] * sum;
    }
  }
};

constexpr int kNT = 24;  // tensor rule of the accepted squares
struct PointRules {
  std::vector<double> gtx, gtw, g12x, g12w;
  LogRule16 R;
  PointRules() {
    gauss_legendre(kNT, gtx, gtw);
    gauss_legendre(12, g12x, g12w);
  }
};


void moment_rules(MomentRules* R) {
  static const PointRules Q;
  const Basis& B = basis();
  for (int i = 0; i < kP; ++i) { R->t[i] = B.t[i]; R->lam[i] = B.lam[i]; R->w[i] = B.w[i]; }
  for (int a = 0; a < kNT; ++a) { R->gx[a] = Q.gtx[size_t(a)]; R->gw[a] = Q.gtw[size_t(a)]; }
  for (int a = 0; a < 12; ++a) { R->px[a] = Q.g12x[size_t(a)]; R->pw[a] = Q.g12w[size_t(a)]; }
  for (int j = 0; j < 16; ++j) { R->u[j] = Q.R.u[j]; R->uw[j] = Q.R.w[j]; R->ul[j] = Q.R.wl[j]; }
}

// D4 element g: (x, y) -> (sx * (swap ? y : x), sy * (swap ? x : y))
struct D4 { int sx, sy, swap; };
static void apply_d4(const D4& g, double x, double y, double& ox, double& oy) {
  double a = g.swap ? y : x, b = g.swap ? x : y;
  ox = g.sx * a;
  oy = g.sy * b;
}
static int node_map(const D4& g, int m) {
  int i = m % kP, j = m / kP;
  int a = g.swap ? j : i, b = g.swap ? i : j;
  int ni = g.sx > 0 ? a : kP - 1 - a, nj = g.sy > 0 ? b : kP - 1 - b;
  return nj * kP + ni;
}

static std::vector<std::vector<double>> near_tables_compute() {
  const auto& NO = near_offsets();
  const Basis& B = basis();
  const int reps[7][3] = {{0, 0, 2}, {4, 0, 2}, {4, 4, 2}, {3, 1, 1}, {3, 3, 1}, {6, 2, 4}, {6, 6, 4}};  // (2dx, 2dy, 2rho)
  std::vector<std::vector<double>> rep(7, std::vector<double>(kNP * kNP));
  std::vector<std::pair<int, int>> jobs;
  for (int r = 0; r < 7; ++r)
    for (int m = 0; m < kNP; ++m) jobs.push_back({r, m});
  unsigned nth = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  std::atomic<size_t> next{0};
  for (unsigned t = 0; t < nth; ++t)
    th.emplace_back([&]() {
      double I[kNP];
      for (;;) {
        size_t id = next.fetch_add(1);
        if (id >= jobs.size()) break;
        int r = jobs[id].first, m = jobs[id].second;
        double dx = 0.5 * reps[r][0], dy = 0.5 * reps[r][1], rho = 0.5 * reps[r][2];
        double xm = B.t[m % kP], ym = B.t[m / kP];
        logint((xm - dx) / rho, (ym - dy) / rho, I);
        double lr = std::log(rho);
        for (int k = 0; k < kNP; ++k) rep[r][size_t(m) * kNP + k] = -kInv2Pi * (lr * B.W[k] + I[k]);
      }
    });
  for (auto& t : th) t.join();
  std::vector<std::vector<double>> out(NO.size());
  const D4 G[8] = {{1, 1, 0}, {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0}, {1, 1, 1}, {-1, 1, 1}, {1, -1, 1}, {-1, -1, 1}};
  for (size_t r = 0; r < NO.size(); ++r) {
    bool done = false;
    for (int q = 0; q < 7 && !done; ++q) {
      double rdx = 0.5 * reps[q][0], rdy = 0.5 * reps[q][1], rrho = 0.5 * reps[q][2];
      if (std::fabs(rrho - NO[r].rho) > 1e-12) continue;
      for (const D4& g : G) {
        double ox, oy;
        apply_d4(g, rdx, rdy, ox, oy);
        if (std::fabs(ox - NO[r].dx) < 1e-12 && std::fabs(oy - NO[r].dy) < 1e-12) {
          out[r].assign(kNP * kNP, 0.0);
          for (int m = 0; m < kNP; ++m)
            for (int k = 0; k < kNP; ++k) out[r][size_t(node_map(g, m)) * kNP + node_map(g, k)] = rep[q][size_t(m) * kNP + k];
          done = true;
          break;
        }
      }
    }
    if (!done) throw std::runtime_error("no D4 representative for a near relation");
  }
  return out;
}

// ---------------------------------------------------------------- cache
static std::string g_cache_dir;
static std::mutex g_cache_mu;
void set_table_cache_dir(const char* dir) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache_dir = dir ? dir : "";
}

static uint64_t fnv1a(const double* d, size_t n) {
  uint64_t h = 1469598103934665603ull;
  const unsigned char* p = reinterpret_cast<const unsigned char*>(d);
  for (size_t i = 0; i < n * sizeof(double); ++i) { h ^= p[i]; h *= 1099511628211ull; }
  return h;
}

static const char kMagic[8] = {'V', 'P', 'N', 'E', 'A', 'R', '0', '1'};

static bool cache_load(const std::string& path, std::vector<std::vector<double>>& out) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  char mg[8];
  int32_t hdr[4];
  uint64_t hash;
  f.read(mg, 8);
  f.read(reinterpret_cast<char*>(hdr), sizeof(hdr));
  f.read(reinterpret_cast<char*>(&hash), 8);
  if (!f || std::memcmp(mg, kMagic, 8) != 0 || hdr[0] != kP || hdr[1] != 33 || hdr[2] != kNP) return false;
  std::vector<double> all(size_t(33) * kNP * kNP);
  f.read(reinterpret_cast<char*>(all.data()), all.size() * sizeof(double));
  if (!f || fnv1a(all.data(), all.size()) != hash) return false;
  out.assign(33, std::vector<double>());
  for (int r = 0; r < 33; ++r) out[r].assign(all.begin() + size_t(r) * kNP * kNP, all.begin() + size_t(r + 1) * kNP * kNP);
  return true;
}

static void cache_store(const std::string& path, const std::vector<std::vector<double>>& t) {
  std::vector<double> all;
  for (auto& v : t) all.insert(all.end(), v.begin(), v.end());
  int32_t hdr[4] = {kP, 33, kNP, 0};
  uint64_t hash = fnv1a(all.data(), all.size());
  std::string tmp = path + ".tmp";
  std::ofstream f(tmp, std::ios::binary);
  if (!f) return;
  f.write(kMagic, 8);
  f.write(reinterpret_cast<const char*>(hdr), sizeof(hdr));
  f.write(reinterpret_cast<const char*>(&hash), 8);
  f.write(reinterpret_cast<const char*>(all.data()), all.size() * sizeof(double));
  f.close();
  if (f) std::rename(tmp.c_str(), path.c_str());
}

// ---------------------------------------------------------------- far-field matrices
static void real_from_linear(const std::vector<cd>& K, int rows, int cols, std::vector<double>& R) {
  // complex-linear map on interleaved (Re, Im)
  R.assign(size_t(2 * rows) * (2 * cols), 0.0);
  for (int l = 0; l < rows; ++l)
    for (int k = 0; k < cols; ++k) {
      cd z = K[size_t(l) * cols + k];
      R[size_t(2 * l) * (2 * cols) + 2 * k] = z.real();
      R[size_t(2 * l) * (2 * cols) + 2 * k + 1] = -z.imag();
      R[size_t(2 * l + 1) * (2 * cols) + 2 * k] = z.imag();
      R[size_t(2 * l + 1) * (2 * cols) + 2 * k + 1] = z.real();
    }
}
static void real_from_realin(const std::vector<cd>& S, int rows, int cols, std::vector<double>& R) {
  // real input (cols) -> complex output (rows)
  R.assign(size_t(2 * rows) * cols, 0.0);
  for (int l = 0; l < rows; ++l)
    for (int k = 0; k < cols; ++k) {
      R[size_t(2 * l) * cols + k] = S[size_t(l) * cols + k].real();
      R[size_t(2 * l + 1) * cols + k] = S[size_t(l) * cols + k].imag();
    }
}
static void real_from_realout(const std::vector<cd>& L, int rows, int cols, std::vector<double>& R) {
  // complex input (cols) -> real output Re(L x) (rows)
  R.assign(size_t(rows) * (2 * cols), 0.0);
  for (int m = 0; m < rows; ++m)
    for (int l = 0; l < cols; ++l) {
      R[size_t(m) * (2 * cols) + 2 * l] = L[size_t(m) * cols + l].real();
      R[size_t(m) * (2 * cols) + 2 * l + 1] = -L[size_t(m) * cols + l].imag();
    }
}
static double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  return std::exp(std::lgamma(n + 1.0) - std::lgamma(k + 1.0) - std::lgamma(n - k + 1.0));
}
static double binom_exact(int n, int k) {
  // Pascal recursion in double: exact below 2^53, correctly rounded-ish above
  static std::vector<std::vector<double>> T;
  if (T.empty()) {
    T.assign(2 * kTerms + 2, std::vector<double>(2 * kTerms + 2, 0.0));
    for (int a = 0; a < int(T.size()); ++a) {
      T[a][0] = 1.0;
      for (int b = 1; b <= a; ++b) T[a][b] = T[a - 1][b - 1] + (b <= a - 1 ? T[a - 1][b] : 0.0);
    }
  }
  if (k < 0 || k > n || n >= int(T.size())) return binom(n, k);
  return T[n][k];
}

// integrals over the reference square of l_k(eta) g(eta) with a tensor Gauss rule of n points
template <class F>
static std::vector<cd> quad_basis(int n, int nfun, F g) {
  std::vector<double> x, w;
  gauss_legendre(n, x, w);
  const Basis& B = basis();
  std::vector<std::vector<double>> L(n, std::vector<double>(kP));
  for (int a = 0; a < n; ++a) B.lagrange(x[a], L[a].data());
  std::vector<cd> out(size_t(nfun) * kNP, cd(0.0));
  std::vector<cd> G(size_t(n) * n);
  for (int f = 0; f < nfun; ++f) {
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) G[size_t(a) * n + b] = w[a] * w[b] * g(f, cd(x[a], x[b]));
    for (int i = 0; i < kP; ++i) {
      std::vector<cd> Cb(n, cd(0.0));
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) Cb[b] += L[a][i] * G[size_t(a) * n + b];
      for (int j = 0; j < kP; ++j) {
        cd s(0.0);
        for (int b = 0; b < n; ++b) s += Cb[b] * L[b][j];
        out[size_t(f) * kNP + j * kP + i] = s;
      }
    }
  }
  return out;
}

// the near tables: the same for every expansion order, computed (or read from the cache) once
static const std::vector<std::vector<double>>& near_tables() {
  static std::once_flag once;
  static std::vector<std::vector<double>>* T = nullptr;
  std::call_once(once, []() {
    T = new std::vector<std::vector<double>>();
    std::string path;
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      if (!g_cache_dir.empty()) path = g_cache_dir + "/volpot_near_p16_v1.bin";
    }
    if (path.empty() || !cache_load(path, *T)) {
      *T = near_tables_compute();
      if (!path.empty()) cache_store(path, *T);
    }
  });
  return *T;
}

// T (n x n, row-major) ~= Q R with Q (n x k, orthonormal columns) and R (k x n): Householder QR
// with column pivoting (the column of largest remaining norm first), stopped after k columns;
// R's columns are returned in T's original order. The discarded part is the trailing block
// R[k:, k:] of the pivoted factorization.
static void pivoted_qr(const std::vector<double>& T, int n, int k, std::vector<double>& Qk, std::vector<double>& Rk) {
  std::vector<double> A(T);
  std::vector<int> perm(static_cast<size_t>(n));
  for (int c = 0; c < n; ++c) perm[size_t(c)] = c;
  std::vector<std::vector<double>> V(static_cast<size_t>(k));
  std::vector<double> beta(static_cast<size_t>(k), 0.0);
  for (int j = 0; j < k; ++j) {
    int p = j;
    double best = -1.0;
    for (int c = j; c < n; ++c) {
      double sq = 0.0;
      for (int i = j; i < n; ++i) sq += A[size_t(i) * n + c] * A[size_t(i) * n + c];
      if (sq > best) { best = sq; p = c; }
    }
    if (p != j) {
      for (int i = 0; i < n; ++i) std::swap(A[size_t(i) * n + j], A[size_t(i) * n + p]);
      std::swap(perm[size_t(j)], perm[size_t(p)]);
    }
    std::vector<double>& v = V[size_t(j)];
    v.assign(size_t(n - j), 0.0);
    double nrm = 0.0;
    for (int i = j; i < n; ++i) { v[size_t(i - j)] = A[size_t(i) * n + j]; nrm += v[size_t(i - j)] * v[size_t(i - j)]; }
    nrm = std::sqrt(nrm);
    const double alpha = v[0] >= 0.0 ? -nrm : nrm;
    v[0] -= alpha;
    double vv = 0.0;
    for (double x : v) vv += x * x;
    beta[size_t(j)] = vv > 0.0 ? 2.0 / vv : 0.0;
    for (int c = j; c < n; ++c) {  // A[j:, c] -= beta v (v . A[j:, c])
      double d = 0.0;
      for (int i = j; i < n; ++i) d += v[size_t(i - j)] * A[size_t(i) * n + c];
      d *= beta[size_t(j)];
      for (int i = j; i < n; ++i) A[size_t(i) * n + c] -= d * v[size_t(i - j)];
    }
  }
  Rk.assign(size_t(k) * n, 0.0);
  for (int i = 0; i < k; ++i)
    for (int c = i; c < n; ++c) Rk[size_t(i) * n + perm[size_t(c)]] = A[size_t(i) * n + c];
  Qk.assign(size_t(n) * k, 0.0);  // H_0 H_1 ... H_{k-1} applied to the first k unit vectors
  for (int c = 0; c < k; ++c) Qk[size_t(c) * k + c] = 1.0;
  for (int j = k - 1; j >= 0; --j) {
    const std::vector<double>& v = V[size_t(j)];
    for (int c = 0; c < k; ++c) {
      double d = 0.0;
      for (int i = j; i < n; ++i) d += v[size_t(i - j)] * Qk[size_t(i) * k + c];
      d *= beta[size_t(j)];
      for (int i = j; i < n; ++i) Qk[size_t(i) * k + c] -= d * v[size_t(i - j)];
    }
  }
}

// The low-rank factors of the 32 adjacent-leaf tables other than the self table, computed once
// (the near tables are the same for every expansion order).
struct NearFactors {
  std::vector<std::vector<double>> U, V;  // 32 each: 256 x k_r and k_r x 256
  std::vector<int> rank;                  // k_r
};
// Truncating a relation's factors after kNearRankLow columns is kept when the discarded part
// is below this fraction of the self table (Frobenius norms). For the 32 relations the
// truncation error is either at rounding level (about 3e-15 of it) or above 1e-11: the
// threshold sits between the two groups.
constexpr double kNearRankLowTol = 1e-13;
static const NearFactors& near_factors() {
  static std::once_flag once;
  static NearFactors* F = nullptr;
  std::call_once(once, []() {
    F = new NearFactors();
    const std::vector<std::vector<double>>& T = near_tables();
    F->U.resize(32);
    F->V.resize(32);
    F->rank.assign(32, kNearRank);
    double self2 = 0.0;
    for (double x : T[0]) self2 += x * x;
    std::vector<std::thread> th;
    for (int r = 1; r <= 32; ++r)
      th.emplace_back([&, r, self2]() {
        std::vector<double>& U = F->U[size_t(r - 1)];
        std::vector<double>& V = F->V[size_t(r - 1)];
        pivoted_qr(T[size_t(r)], kNP, kNearRank, U, V);
        const int k = kNearRankLow;
        double e2 = 0.0;  // || T_r - U_r[:, :k] V_r[:k, :] ||_F^2
        for (int i = 0; i < kNP; ++i)
          for (int j = 0; j < kNP; ++j) {
            double s = T[size_t(r)][size_t(i) * kNP + j];
            for (int c = 0; c < k; ++c) s -= U[size_t(i) * kNearRank + c] * V[size_t(c) * kNP + j];
            e2 += s * s;
          }
        if (e2 > kNearRankLowTol * kNearRankLowTol * self2) return;
        std::vector<double> Uk(size_t(kNP) * k);
        for (int i = 0; i < kNP; ++i)
          for (int c = 0; c < k; ++c) Uk[size_t(i) * k + c] = U[size_t(i) * kNearRank + c];
        U.swap(Uk);
        V.resize(size_t(k) * kNP);  // the first k rows
        F->rank[size_t(r - 1)] = k;
      });
    for (auto& t : th) t.join();
  });
  return *F;
}

static Matrices build_matrices(const int Q) {
  const int kNE = 2 * Q;  // reals per expansion for this order
  Matrices M;
  M.M.assign(kNumRel, 0);
  M.K.assign(kNumRel, 0);
  M.a.assign(kNumRel, {});
  M.nnz.assign(kNumRel, 0.0);
  M.w_in.assign(kNumRel, {});
  M.w_out.assign(kNumRel, {});
  M.lnd.assign(kNumRel, 0.0);
  M.koff.assign(kNumRel, 0);
  const Basis& B = basis();
  std::vector<cd> xi(kNP);
  for (int m = 0; m < kNP; ++m) xi[m] = cd(B.t[m % kP], B.t[m / kP]);
  auto set = [&](int id, int rows, int cols, std::vector<double>&& a) {
    M.M[id] = rows; M.K[id] = cols; M.a[id] = std::move(a);
  };
  // S2M: c_n int l_k eta^n, c_0 = 1, c_n = -1/n
  {
    auto S = quad_basis(40, Q, [](int n, cd e) { return n == 0 ? cd(1.0) : -std::pow(e, n) / double(n); });
    std::vector<double> R;
    real_from_realin(S, Q, kNP, R);
    set(kRelS2M, kNE, kNP, std::move(R));
  }
  // M2M_q and L2L_q
  for (int q = 0; q < 4; ++q) {
    cd z0((q & 1) ? 0.5 : -0.5, (q & 2) ? 0.5 : -0.5);
    std::vector<cd> Bm(size_t(Q) * Q, cd(0.0)), E(size_t(Q) * Q, cd(0.0));
    Bm[0] = 1.0;
    for (int l = 1; l < Q; ++l) {
      Bm[size_t(l) * Q] = -std::pow(z0, l) / double(l);
      for (int k = 1; k <= l; ++k) Bm[size_t(l) * Q + k] = std::ldexp(1.0, -k) * binom_exact(l - 1, k - 1) * std::pow(z0, l - k);
    }
    for (int l = 0; l < Q; ++l)
      for (int k = l; k < Q; ++k) E[size_t(l) * Q + k] = binom_exact(k, l) * std::pow(z0, k - l) * std::ldexp(1.0, -l);
    std::vector<double> R1, R2;
    real_from_linear(Bm, Q, Q, R1);
    real_from_linear(E, Q, Q, R2);
    set(kRelM2M + q, kNE, kNE, std::move(R1));
    set(kRelL2L + q, kNE, kNE, std::move(R2));
  }
  // two-level translations: M2M_qc M2M_qg (grandchild to box) and L2L_qg L2L_qc (box to grandchild)
  for (int qc = 0; qc < 4; ++qc)
    for (int qg = 0; qg < 4; ++qg) {
      std::vector<double> Pm(size_t(kNE) * kNE, 0.0), Pl(size_t(kNE) * kNE, 0.0);
      const std::vector<double>& Mc = M.a[kRelM2M + qc];
      const std::vector<double>& Mg = M.a[kRelM2M + qg];
      const std::vector<double>& Lc = M.a[kRelL2L + qc];
      const std::vector<double>& Lg = M.a[kRelL2L + qg];
      for (int i = 0; i < kNE; ++i)
        for (int k = 0; k < kNE; ++k) {
          const double mc = Mc[size_t(i) * kNE + k], lg = Lg[size_t(i) * kNE + k];
          for (int j = 0; j < kNE; ++j) {
            Pm[size_t(i) * kNE + j] += mc * Mg[size_t(k) * kNE + j];
            Pl[size_t(i) * kNE + j] += lg * Lc[size_t(k) * kNE + j];
          }
        }
      set(kRelM2M2 + 4 * qc + qg, kNE, kNE, std::move(Pm));
      set(kRelL2L2 + 4 * qc + qg, kNE, kNE, std::move(Pl));
    }
  // M2L_r: d = (source - target centre) / s
  const auto& VO = v_offsets();
  for (size_t r = 0; r < VO.size(); ++r) {
    cd d(VO[r].dx, VO[r].dy);
    std::vector<cd> K(size_t(Q) * Q, cd(0.0));
    K[0] = std::log(std::abs(d));
    for (int k = 1; k < Q; ++k) K[k] = ((k & 1) ? -1.0 : 1.0) * std::pow(d, -k);
    for (int l = 1; l < Q; ++l) {
      K[size_t(l) * Q] = -1.0 / (double(l) * std::pow(d, l));
      for (int k = 1; k < Q; ++k) K[size_t(l) * Q + k] = ((k & 1) ? -1.0 : 1.0) * binom_exact(k + l - 1, l) * std::pow(d, -(k + l));
    }
    std::vector<double> R;
    real_from_linear(K, Q, Q, R);
    set(kRelM2L + int(r), kNE, kNE, std::move(R));
    // the same map factored: w_out = d^-l, w_in = (-1)^k d^-k around the core kRelH; the
    // adjoint (the real transpose) conjugates both diagonals and swaps their roles
    const int id = kRelM2L + int(r), ia = id + kNumFwd, QP = pad16(Q);
    M.w_in[id].assign(size_t(2 * Q), 0.0);
    M.w_out[id].assign(size_t(2 * QP), 0.0);
    M.w_in[ia].assign(size_t(2 * Q), 0.0);
    M.w_out[ia].assign(size_t(2 * QP), 0.0);
    for (int k = 0; k < Q; ++k) {
      const cd dl = std::pow(d, -k), dr = ((k & 1) ? -1.0 : 1.0) * dl;
      M.w_out[id][size_t(2 * k)] = dl.real(); M.w_out[id][size_t(2 * k + 1)] = dl.imag();
      M.w_in[id][size_t(2 * k)] = dr.real(); M.w_in[id][size_t(2 * k + 1)] = dr.imag();
      M.w_in[ia][size_t(2 * k)] = dl.real(); M.w_in[ia][size_t(2 * k + 1)] = -dl.imag();
      M.w_out[ia][size_t(2 * k)] = dr.real(); M.w_out[ia][size_t(2 * k + 1)] = -dr.imag();
    }
    M.lnd[id] = M.lnd[ia] = std::log(std::abs(d));
  }
  {  // the offset-free core of the factored M2L, rows padded to a multiple of 16
    const int QP = pad16(Q);
    std::vector<double> H(size_t(QP) * Q, 0.0);
    for (int k = 1; k < Q; ++k) H[size_t(k)] = 1.0;
    for (int l = 1; l < Q; ++l) {
      H[size_t(l) * Q] = -1.0 / double(l);
      for (int k = 1; k < Q; ++k) H[size_t(l) * Q + k] = binom_exact(k + l - 1, l);
    }
    set(kRelH, QP, Q, std::move(H));
  }
  // S2L_r: source leaf (rho = 2) at d = (source - target centre) / s_target
  const auto& XO = x_offsets();
  for (size_t r = 0; r < XO.size(); ++r) {
    cd d(XO[r].dx, XO[r].dy);
    double rho = XO[r].rho;
    auto S = quad_basis(48, Q, [&](int l, cd e) {
      cd w = d + rho * e;
      return l == 0 ? cd(std::log(std::abs(w))) : -std::pow(w, -l) / double(l);
    });
    std::vector<double> R;
    real_from_realin(S, Q, kNP, R);
    set(kRelS2L + int(r), kNE, kNP, std::move(R));
  }
  // near tables
  {
    const std::vector<std::vector<double>>& T = near_tables();
    for (int r = 0; r < 33; ++r) set(kRelNear + r, kNP, kNP, std::vector<double>(T[size_t(r)]));
    // the low-rank form of relations 1..32 and the 64-column slices of the self table
    const NearFactors& F = near_factors();
    for (int r = 0; r < 32; ++r) {
      const int k = F.rank[size_t(r)];
      set(kRelNU + r, kNP, k, std::vector<double>(F.U[size_t(r)]));
      set(kRelNV + r, k, kNP, std::vector<double>(F.V[size_t(r)]));
    }
    const std::vector<double>& S = T[0];
    for (int q = 0; q < 4; ++q) {
      std::vector<double> fw(size_t(kNP) * 64), ad(size_t(kNP) * 64);
      for (int i = 0; i < kNP; ++i)
        for (int c = 0; c < 64; ++c) {
          fw[size_t(i) * 64 + c] = S[size_t(i) * kNP + 64 * q + c];  // T[i][64q + c]
          ad[size_t(i) * 64 + c] = S[size_t(64 * q + c) * kNP + i];  // (T[64q + c][i]): T^T's column block
        }
      set(kRelNSF + q, kNP, 64, std::move(fw));
      set(kRelNSA + q, kNP, 64, std::move(ad));
      M.koff[size_t(kRelNSF + q)] = M.koff[size_t(kRelNSA + q)] = 64 * q;
    }
  }
  // M2T_r: source box (rho = 1/2) at d = (source - target centre) / s_target
  const auto& WO = w_offsets();
  for (size_t r = 0; r < WO.size(); ++r) {
    cd d(WO[r].dx, WO[r].dy);
    double rho = WO[r].rho;
    std::vector<cd> Mt(size_t(kNP) * Q);
    for (int m = 0; m < kNP; ++m) {
      cd z = xi[m] - d;
      Mt[size_t(m) * Q] = -kInv2Pi * std::log(std::abs(z));
      for (int k = 1; k < Q; ++k) Mt[size_t(m) * Q + k] = -kInv2Pi * std::pow(rho, k) * std::pow(z, -k);
    }
    std::vector<double> R;
    real_from_realout(Mt, kNP, Q, R);
    set(kRelM2T + int(r), kNP, kNE, std::move(R));
  }
  // L2T
  {
    std::vector<cd> Lt(size_t(kNP) * Q);
    for (int m = 0; m < kNP; ++m)
      for (int l = 0; l < Q; ++l) Lt[size_t(m) * Q + l] = -kInv2Pi * std::pow(xi[m], l);
    std::vector<double> R;
    real_from_realout(Lt, kNP, Q, R);
    set(kRelL2T, kNP, kNE, std::move(R));
  }
  // transposes
  for (int id = 0; id < kNumFwd; ++id) {
    int r = M.M[id], c = M.K[id];
    std::vector<double> T(size_t(r) * c);
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < c; ++j) T[size_t(j) * r + i] = M.a[id][size_t(i) * c + j];
    set(id + kNumFwd, c, r, std::move(T));
  }
  {  // the core's transpose keeps the padded shape: rows k (padded), columns l
    const int QP = pad16(Q);
    const std::vector<double>& H = M.a[kRelH];
    std::vector<double> T(size_t(QP) * Q, 0.0);
    for (int l = 0; l < Q; ++l)
      for (int k = 0; k < Q; ++k) T[size_t(k) * Q + l] = H[size_t(l) * Q + k];
    set(kRelH + kNumFwd, QP, Q, std::move(T));
  }
  for (int id = 0; id < kNumRel; ++id) {
    double n = 0;
    for (double v : M.a[id]) n += (v != 0.0);
    M.nnz[id] = n;
  }
  return M;
}

const Matrices& matrices(int q) {
  static std::mutex mu;
  static std::map<int, const Matrices*> built;
  std::lock_guard<std::mutex> lk(mu);
  auto it = built.find(q);
  if (it == built.end()) it = built.emplace(q, new Matrices(build_matrices(q))).first;
  return *it->second;
}

}  // namespace vp
