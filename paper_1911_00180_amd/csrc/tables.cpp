// Host-side tables of the worm-LBM (see tables.hpp).
#include "tables.hpp"

#include <algorithm>

#include <cmath>
#include <cstdlib>
#include <stdexcept>

namespace wlbm {

namespace {

constexpr double kTwoPi = 2.0 * M_PI;

// Sum with a running compensation term (Neumaier) so that Lambda_corr does
// not depend on the order of the directions beyond the last bit.
double compensated_sum(const std::vector<double>& v) {
  double s = 0.0, c = 0.0;
  for (double x : v) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  return s + c;
}

void fill_octant(DirSet& d, int i, double ax, double ay) {
  // ax, ay: the components that decide the octant (exact integers for the
  // ring set, the FP64 unit vector for the uniform set)
  const int mj = (std::fabs(ax) >= std::fabs(ay)) ? 0 : 1;
  const double big = mj == 0 ? ax : ay;
  const double small = mj == 0 ? ay : ax;
  d.major[i] = mj;
  d.sgn_major[i] = big > 0 ? 1 : -1;
  d.sgn_minor[i] = small > 0 ? 1 : (small < 0 ? -1 : 0);
}

}  // namespace

DirSet build_dirs(int q, int kind) {
  if (q < 8 || q % 8 != 0) throw std::invalid_argument("q must be a positive multiple of 8");
  DirSet d;
  d.q = q;
  d.kind = kind;
  d.m = q / 8;
  d.sx.assign(q, 0.0);
  d.sy.assign(q, 0.0);
  d.w.assign(q, 0.0);
  d.speed.assign(q, 0.0);
  d.slope.assign(q, 0.0);
  d.major.assign(q, 0);
  d.sgn_major.assign(q, 0);
  d.sgn_minor.assign(q, 0);
  d.ring_j.assign(q, 0);

  if (kind == kUniform) {
    // theta_i = 2 pi i / Q.  On the axes and diagonals (8i/Q integer) the
    // exact unit vectors are used, so these worms are exact axial/diagonal.
    const double r2 = std::sqrt(0.5);
    const double ex[8][2] = {{1.0, 0.0}, {r2, r2},   {0.0, 1.0},  {-r2, r2},
                             {-1.0, 0.0}, {-r2, -r2}, {0.0, -1.0}, {r2, -r2}};
    for (int i = 0; i < q; ++i) {
      double cx, cy;
      if ((8 * i) % q == 0) {
        cx = ex[(8 * i) / q][0];
        cy = ex[(8 * i) / q][1];
      } else {
        const double theta = 2.0 * M_PI * i / q;
        cx = std::cos(theta);
        cy = std::sin(theta);
      }
      d.sx[i] = cx;
      d.sy[i] = cy;
      fill_octant(d, i, cx, cy);
      const double big = std::fabs(d.major[i] == 0 ? cx : cy);
      const double small = std::fabs(d.major[i] == 0 ? cy : cx);
      d.slope[i] = small / big;
      d.speed[i] = 1.0 / big;
      d.w[i] = 1.0 / q;
    }
  } else if (kind == kRing) {
    // The 8M lattice vectors of the square ring max(|x|,|y|) = M, walked
    // counter-clockwise starting at (M, 0).
    const int M = d.m;
    std::vector<int> vx, vy;
    vx.reserve(q);
    vy.reserve(q);
    for (int j = 0; j < M; ++j) { vx.push_back(M); vy.push_back(j); }
    for (int j = 0; j < 2 * M; ++j) { vx.push_back(M - j); vy.push_back(M); }
    for (int j = 0; j < 2 * M; ++j) { vx.push_back(-M); vy.push_back(M - j); }
    for (int j = 0; j < 2 * M; ++j) { vx.push_back(-M + j); vy.push_back(-M); }
    for (int j = 0; j < M; ++j) { vx.push_back(M); vy.push_back(-M + j); }
    std::vector<double> phi(q);
    for (int i = 0; i < q; ++i) {
      const double len = std::hypot(double(vx[i]), double(vy[i]));
      d.sx[i] = vx[i] / len;
      d.sy[i] = vy[i] / len;
      fill_octant(d, i, vx[i], vy[i]);
      const int big = std::abs(d.major[i] == 0 ? vx[i] : vy[i]);
      const int small = std::abs(d.major[i] == 0 ? vy[i] : vx[i]);
      (void)big;
      d.ring_j[i] = small;
      d.slope[i] = double(small) / M;
      d.speed[i] = len / M;
      double a = std::atan2(double(vy[i]), double(vx[i]));
      if (a < 0.0) a += kTwoPi;
      phi[i] = a;
    }
    // Eq. weight with the theta's read as angular gaps between neighbours:
    // w_j = (phi_{j+1} - phi_{j-1}) / (4 pi), cyclic.
    for (int j = 0; j < q; ++j) {
      double up = phi[(j + 1) % q] - phi[j];
      if (up < 0.0) up += kTwoPi;
      double dn = phi[j] - phi[(j + q - 1) % q];
      if (dn < 0.0) dn += kTwoPi;
      d.w[j] = (up + dn) / (4.0 * M_PI);
    }
  } else {
    throw std::invalid_argument("unknown direction set");
  }
  d.lambda_corr = q / compensated_sum(d.speed);
  d.vgrid.assign(q, 1.0);
  // mirror image in a y wall (Eq. adiabatic-specular): both sets are
  // symmetric under (sx, sy) -> (sx, -sy)
  d.mirror_y.assign(q, -1);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j)
      if (std::fabs(d.sx[j] - d.sx[i]) < 1e-12 && std::fabs(d.sy[j] + d.sy[i]) < 1e-12)
        d.mirror_y[i] = j;
  for (int i = 0; i < q; ++i)
    if (d.mirror_y[i] < 0) throw std::invalid_argument("direction set without y mirror pairs");
  return d;
}

double corrected_weight(double W, double lambda_corr, bool emulate_3d, bool correction) {
  if (!correction) return W;
  const double f = emulate_3d ? 1.5 : 1.0;
  return f * ((1.0 - W) * W + W * (W * lambda_corr));
}

int64_t worm_minor(const DirSet& d, int i, int64_t k) {
  if (k <= 0) return 0;
  if (d.kind == kRing) {
    const int64_t M = d.m;
    return (2 * k * d.ring_j[i] + M) / (2 * M);
  }
  const double f = double(k) * d.slope[i];
  const double fl = std::floor(f);
  return int64_t(fl) + ((f - fl) >= 0.5 ? 1 : 0);
}

void worm_move(const DirSet& d, int i, int64_t k, int* dx, int* dy) {
  const int step_minor = int(worm_minor(d, i, k) - worm_minor(d, i, k - 1)) * d.sgn_minor[i];
  if (d.major[i] == 0) {
    *dx = d.sgn_major[i];
    *dy = step_minor;
  } else {
    *dx = step_minor;
    *dy = d.sgn_major[i];
  }
}

int d2q8_index(int dx, int dy) {
  static const int table[3][3] = {
      // dy = -1, 0, +1  for dx = -1
      {7, 3, 6},
      // dx = 0
      {4, 0, 2},
      // dx = +1
      {8, 1, 5}};
  return table[dx + 1][dy + 1];
}

void TasState::reset(int q) {
  px.assign(q, 0);
  py.assign(q, 0);
  k.assign(q, 0);
  n = 0;
}

void tas_advance(const DirSet& d, TasState& st, int8_t* dx, int8_t* dy, uint8_t* hop) {
  const int64_t n = st.n + 1;
  const int64_t r = n + 1;
  for (int i = 0; i < d.q; ++i) {
    int mx, my;
    worm_move(d, i, st.k[i] + 1, &mx, &my);
    const int64_t cx = st.px[i] + mx;
    const int64_t cy = st.py[i] + my;
    bool h;
    if (d.vgrid[i] == 1.0) {
      h = cx * cx + cy * cy <= r * r;
    } else {
      const double rv = d.vgrid[i] * double(n) + 1.0;
      h = double(cx * cx + cy * cy) <= rv * rv;
    }
    if (h) {
      st.px[i] = cx;
      st.py[i] = cy;
      st.k[i] += 1;
    }
    dx[i] = int8_t(mx);
    dy[i] = int8_t(my);
    hop[i] = h ? 1 : 0;
  }
  st.n = n;
}

void tas_restore(const DirSet& d, TasState& st, int64_t n, const int32_t* k) {
  st.reset(d.q);
  st.n = n;
  for (int i = 0; i < d.q; ++i) {
    const int64_t kk = k[i];
    const int64_t major = kk * d.sgn_major[i];
    const int64_t minor = worm_minor(d, i, kk) * d.sgn_minor[i];
    st.k[i] = kk;
    st.px[i] = d.major[i] == 0 ? major : minor;
    st.py[i] = d.major[i] == 0 ? minor : major;
  }
}

void ScheduleBook::reset(const DirSet* d) {
  d_ = d;
  snaps_.assign(1, std::vector<int32_t>(d->q, 0));
}

void ScheduleBook::note(const TasState& st) {
  if (st.n % kSnapEvery != 0) return;
  const int64_t s = st.n / kSnapEvery;
  if (s != int64_t(snaps_.size())) return;
  std::vector<int32_t> k(d_->q);
  for (int i = 0; i < d_->q; ++i) k[i] = int32_t(st.k[i]);
  snaps_.push_back(std::move(k));
}

void ScheduleBook::state_at(int64_t n, TasState& out) {
  int64_t s = std::min<int64_t>(n / kSnapEvery, int64_t(snaps_.size()) - 1);
  tas_restore(*d_, out, s * kSnapEvery, snaps_[size_t(s)].data());
  std::vector<int8_t> dx(d_->q), dy(d_->q);
  std::vector<uint8_t> hop(d_->q);
  while (out.n < n) {
    tas_advance(*d_, out, dx.data(), dy.data(), hop.data());
    note(out);
  }
}

void ScheduleBook::rows(int64_t first, int64_t count, int8_t* dx, int8_t* dy, uint8_t* hop) {
  TasState st;
  state_at(first - 1, st);
  const size_t q = size_t(d_->q);
  for (int64_t r = 0; r < count; ++r) {
    tas_advance(*d_, st, dx + r * q, dy + r * q, hop + r * q);
    note(st);
  }
}

}  // namespace wlbm
