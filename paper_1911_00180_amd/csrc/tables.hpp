// Host-side tables of the worm-LBM: direction sets, angular weights, the
// grid-MFP correction, closed-form worm paths and the integer TAS schedule.
// Plain C++17, no GPU code; used by the C-ABI layer to build what the kernels
// read.  Sections and equations are those of arXiv:1911.00180.
#pragma once

#include <cstdint>
#include <vector>

namespace wlbm {

enum DirKind { kUniform = 0, kRing = 1 };

// One direction set D2Q[M x 8] (Sec. 2.4).  For each direction i:
//   sx, sy      unit vector
//   w           angular weight (Eq. weight; 1/Q for the uniform set)
//   speed       net displacement of one worm hop, c_i = 1/max(|sx|,|sy|)
//   major       axis of the larger component (0 = x, 1 = y; the diagonals,
//               where both are equal, take x)
//   sgn_major   sign of the major component (+1/-1)
//   sgn_minor   sign of the minor component (+1/-1, 0 on an axis)
//   slope       |minor| / |major| in FP64 (uniform set)
//   ring_j      |minor| of the integer lattice vector (ring set; |major| = M)
struct DirSet {
  int q = 0;
  int kind = kUniform;
  int m = 0;
  std::vector<double> sx, sy, w, speed, slope;
  std::vector<int> major, sgn_major, sgn_minor;
  std::vector<int> mirror_y;  // index of the direction (sx, -sy)
  std::vector<double> vgrid;  // grid speed in cells per step, (0, 1] (Sec. 2.3)
  std::vector<int64_t> ring_j;
  double lambda_corr = 0.0;  // Q / sum_i speed_i (Eq. W-correction-factor-gereralized)
};

DirSet build_dirs(int q, int kind);

// Corrected relaxation weight of Eq. W-correction; f = 3/2 when a 2D run
// emulates 3D, the plain W when the correction is switched off.
double corrected_weight(double W, double lambda_corr, bool emulate_3d, bool correction);

// Coordinate along the minor axis (in magnitude) of the worm after k hops.
// The worm takes the D2Q8 move whose landing point is nearest to the ray
// point with major coordinate k (Eq. worm-paths), ties going to the diagonal
// move; its minor coordinate is therefore k*t rounded half up.  For the ring
// set t = j/M and the rounding is done in integers.
int64_t worm_minor(const DirSet& d, int i, int64_t k);

// The k-th (1-based) worm move of direction i as a D2Q8 step (dx, dy).
void worm_move(const DirSet& d, int i, int64_t k, int* dx, int* dy);

// D2Q8 index 1..8 (E, N, W, S, NE, NW, SW, SE) of a step (dx, dy).
int d2q8_index(int dx, int dy);

// Time-adaptive scheme state (Sec. 2.3, Sec. 2.5): per direction the worm
// position P_i and the number k_i of executed worm moves; n = steps done.
struct TasState {
  std::vector<int64_t> px, py, k;
  int64_t n = 0;
  void reset(int q);
};

// One step of the schedule (step n = st.n + 1): for each direction the
// pending move s_i and whether the DDED hops, hop iff |P_i + s_i|^2 <= (n+1)^2
// in exact integers; on a hop P_i and k_i advance.  Outputs are [q] arrays.
// A direction with grid speed v_i != 1 hops iff |P_i + s_i|^2 <= (v_i n + 1)^2,
// evaluated in float64 (the axial distance after step n is v_i n).
void tas_advance(const DirSet& d, TasState& st, int8_t* dx, int8_t* dy, uint8_t* hop);

// The state after n steps from the hop counts k_i alone: after k hops the
// worm of direction i sits at k along its major axis and worm_minor(k) along
// its minor axis, with the signs of the direction.
void tas_restore(const DirSet& d, TasState& st, int64_t n, const int32_t* k);

// Schedule rows of any step range, from snapshots of the hop counts taken
// every kSnapEvery steps (4 q bytes each) as the schedule is first produced;
// a range is regenerated from the nearest snapshot at or before it.
class ScheduleBook {
 public:
  static constexpr int64_t kSnapEvery = 64;
  void reset(const DirSet* d);
  // State after `n` steps.
  void state_at(int64_t n, TasState& out);
  // Record the hop counts of `st` if it sits on a snapshot step not yet held.
  void note(const TasState& st);
  // dx/dy/hop of steps first .. first + count - 1 (first >= 1) into
  // [count][q] arrays.
  void rows(int64_t first, int64_t count, int8_t* dx, int8_t* dy, uint8_t* hop);

 private:
  const DirSet* d_ = nullptr;
  std::vector<std::vector<int32_t>> snaps_;  // snaps_[s]: k_i after s * kSnapEvery steps
};

}  // namespace wlbm
