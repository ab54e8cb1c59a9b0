// postsolve.hip -- the host postsolver of libpsl (section 2.1, "Postsolver":
// the reductions are undone from the stack, last first, each mapping a
// solution of the problem after it to one of the problem before it; section
// 3.3: postsolve runs on the CPU and returns primal and dual solutions of
// the original LP).
//
// Organisation: the record stream is indexed once (the values of removed
// columns, the members of every parallel-column group, the lambda of every
// merged row), then a single reverse walk dispatches each record to the
// handler of its type. Handlers touch only the solution vectors and the
// index. The arithmetic each handler performs, and its summation order, is
// the one the library's readings fix, so that the result is reproducible
// bit for bit:
//   * a removed column with FIX_COL / EMPTY_COL / DUAL_FIX holds its recorded
//     value (a constant of the problem from then on);
//   * a free column singleton j of row i takes x_j = (s - rest) / a_ij, rest =
//     the row's other original terms added left to right, s = the recorded
//     side (1: lhs, 2: rhs) or, without a cost (0), rest moved into the
//     recorded sides (below lhs -> lhs, else above rhs -> rhs);
//   * a parallel-column group splits its leader's value: the prefix
//     intervals B_0 = old leader bounds, B_s = B_{s-1} + lambda_s [lb_s, ub_s]
//     (lambda < 0 swaps the ends; |v| >= inf_value -> +-inf, -0 -> +0) are
//     rebuilt in member order, and members, last first, take the point of
//     [lb_s, ub_s] that keeps the remainder in B_{s-1}, starting from lb_s if
//     finite, else ub_s, else 0, moved into that range (below -> its low end,
//     else above -> its high end); the leader keeps the remainder;
//   * a doubleton substitution gives the eliminated column x_k =
//     (b - a_j x_j) / a_k;
//   * dual: kept rows take the reduced duals, the others start at 0; a
//     BOUND_CHANGE whose column carries a multiplier of its bound's sign
//     (z_j = c_j - a_j'y, summed over the input's column j ascending, left to
//     right) passes it to its source row k: y_k += z_j / a_kj; an active merged
//     side of a parallel-row leader (y_L > 0: lhs, < 0: rhs) goes back to the
//     row r that gave it, y_r = y_L / lambda_r, y_L = 0; a FREE_SINGLETON row
//     has y_i = c_j / a_ij from the start of the pass (the costs of the
//     problems after it include -y_i a_ik); a DOUBLETON_ROW adds to its row the multiplier
//     that makes z_k = c_k - a_k'y zero (c_k the cost then, the sum over the
//     input's column k without row i): Y = (c_k - sum) / a_k. Until that record
//     is undone, the reduced cost of its kept column j is taken in the problem
//     of that time, whose rows of k were rewritten by -f_r row_i and whose
//     cost lost (c_k / a_k) a_j: z_j - a_j Y. Finally z = c - A'y.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <unordered_map>
#include <vector>

#include "engine.h"

namespace psl {
namespace {

// Record types the postsolver reads (the numbering of the C-ABI's record
// documentation in psl.h).
enum : uint8_t {
  T_FIX_COL = 1, T_EMPTY_COL = 2, T_BOUND_CHANGE = 6, T_PARALLEL_ROW = 7, T_LEADER_SIDES = 8,
  T_DUAL_FIX = 9, T_FREE_SINGLETON = 10, T_PARALLEL_COL = 11, T_LEADER_BOUNDS = 12, T_DOUBLETON_ROW = 14,
  T_DOMINATED_COL = 15
};

// value of a merged interval end under the library's infinity convention
inline double interval_end(double v, double inf_value) {
  if (std::fabs(v) >= inf_value) return std::copysign(HUGE_VAL, v);
  return v == 0.0 ? 0.0 : v;
}

// x moved into [lo, hi]: below lo gives lo, otherwise above hi gives hi
inline double move_into(double x, double lo, double hi) {
  if (x < lo) return lo;
  if (x > hi) return hi;
  return x;
}

// A group of merged parallel columns: the leader, its bounds before the
// merge, and the members in the order the merge added them.
struct ColumnGroup {
  int32_t leader = -1;
  double low0 = 0.0, high0 = 0.0;
  struct Member {
    int32_t col;
    double lambda, lb, ub;
  };
  std::vector<Member> members;

  // x[leader] holds the merged variable's value; give every member its share
  void split(double inf_value, double* x) const {
    size_t cnt = members.size();
    // prefix intervals, B[0] the leader's own
    std::vector<double> low(cnt + 1), high(cnt + 1);
    low[0] = low0;
    high[0] = high0;
    for (size_t s = 1; s <= cnt; ++s) {
      const Member& mb = members[s - 1];
      double add_lo = mb.lambda > 0 ? mb.lambda * mb.lb : mb.lambda * mb.ub;
      double add_hi = mb.lambda > 0 ? mb.lambda * mb.ub : mb.lambda * mb.lb;
      low[s] = interval_end(low[s - 1] + add_lo, inf_value);
      high[s] = interval_end(high[s - 1] + add_hi, inf_value);
    }
    double rest = x[leader];
    for (size_t s = cnt; s >= 1; --s) {
      const Member& mb = members[s - 1];
      // rest - lambda * v must stay within [low[s-1], high[s-1]]
      double from_low = (rest - low[s - 1]) / mb.lambda;
      double from_high = (rest - high[s - 1]) / mb.lambda;
      double a = mb.lambda > 0 ? from_high : from_low;
      double b = mb.lambda > 0 ? from_low : from_high;
      double lo_v = a > mb.lb ? a : mb.lb;  // ties take the bound
      double hi_v = b < mb.ub ? b : mb.ub;
      double start = std::isinf(mb.lb) ? (std::isinf(mb.ub) ? 0.0 : mb.ub) : mb.lb;
      double v = move_into(start, lo_v, hi_v);
      x[mb.col] = v;
      rest = rest - mb.lambda * v;
    }
    x[leader] = rest;
  }
};

// The stream, indexed once.
class RecordStack {
 public:
  RecordStack(const psl_record* rec, int64_t count) : rec_(rec), count_(count) {
    std::unordered_map<int32_t, int64_t> open;  // leader column -> its group's record, this pass
    int32_t pass = -1;
    for (int64_t t = 0; t < count; ++t) {
      const psl_record& r = rec[t];
      switch (r.type) {
        case T_FIX_COL:
        case T_EMPTY_COL:
        case T_DUAL_FIX:
        case T_DOMINATED_COL:
          fixed_.push_back({r.j, r.v[0]});
          break;
        case T_FREE_SINGLETON:
          needs_rows_ = true;
          substituted_.push_back({r.i, r.v[3] / r.v[0]});
          break;
        case T_PARALLEL_ROW:
          row_lambda_[r.i] = r.v[0];
          break;
        case T_DOUBLETON_ROW:
          kept_by_[r.j] = t;
          break;
        case T_LEADER_BOUNDS: {
          if (r.round != pass) {
            open.clear();
            pass = r.round;
          }
          ColumnGroup& g = groups_[t];
          g.leader = r.j;
          g.low0 = r.v[0];
          g.high0 = r.v[1];
          open[r.j] = t;
          break;
        }
        case T_PARALLEL_COL: {
          if (r.round != pass) {
            open.clear();
            pass = r.round;
          }
          auto it = open.find(r.k);
          if (it != open.end()) groups_[it->second].members.push_back({r.j, r.v[0], r.v[1], r.v[2]});
          break;
        }
        default:
          break;
      }
    }
  }

  bool needs_rows() const { return needs_rows_; }

  void primal(double* x, const HostRows* rows, double inf_value) const {
    for (const auto& f : fixed_) x[f.first] = f.second;
    for (int64_t t = count_ - 1; t >= 0; --t) {
      const psl_record& r = rec_[t];
      if (r.type == T_LEADER_BOUNDS) groups_.at(t).split(inf_value, x);
      else if (r.type == T_FREE_SINGLETON) x[r.j] = singleton_value(r, *rows, x);
      else if (r.type == T_DOUBLETON_ROW) x[r.k] = (r.v[2] - r.v[0] * x[r.j]) / r.v[1];
    }
  }

  void dual(const HostCols& A, double* y) {
    // rows substituted into the objective carry their dual in every problem
    // after their removal (the other columns' costs lost y_i a_ik)
    for (const auto& rd : substituted_) y[rd.first] = rd.second;
    for (int64_t t = count_ - 1; t >= 0; --t) {
      const psl_record& r = rec_[t];
      switch (r.type) {
        case T_BOUND_CHANGE:
          undo_tightening(r, A, y);
          break;
        case T_DOUBLETON_ROW:
          y[r.i] = y[r.i] + substitution_dual(r, A, y);
          kept_by_.erase(r.j);
          break;
        case T_LEADER_SIDES:
          undo_merged_sides(r, y);
          break;
        default:
          break;
      }
    }
  }

  static double reduced_cost(const HostCols& A, const double* y, int32_t j) {
    double ay = 0.0;
    for (int32_t q = A.cp[j]; q < A.cp[j + 1]; ++q) ay = ay + A.cva[q] * y[A.ri[q]];
    return A.c[j] - ay;
  }

 private:
  static double singleton_value(const psl_record& r, const HostRows& rows, const double* x) {
    double rest = 0.0;
    for (int32_t q = rows.rp[r.i]; q < rows.rp[r.i + 1]; ++q) {
      int32_t k = rows.ci[q];
      if (k != r.j) rest = rest + rows.va[q] * x[k];
    }
    double s = r.side == 1 ? r.v[1] : (r.side == 2 ? r.v[2] : move_into(rest, r.v[1], r.v[2]));
    return (s - rest) / r.v[0];
  }

  // the multiplier a doubleton substitution's row takes to zero z_k
  static double substitution_dual(const psl_record& r, const HostCols& A, const double* y) {
    double ay = 0.0;
    for (int32_t q = A.cp[r.k]; q < A.cp[r.k + 1]; ++q)
      if (A.ri[q] != r.i) ay = ay + A.cva[q] * y[A.ri[q]];
    return (r.v[3] - ay) / r.v[1];
  }

  // reduced cost of column j in the problem of the record being undone
  double reduced_cost_then(const HostCols& A, const double* y, int32_t j) const {
    double z = reduced_cost(A, y, j);
    auto it = kept_by_.find(j);
    if (it != kept_by_.end()) {
      const psl_record& s = rec_[it->second];
      z = z - s.v[0] * substitution_dual(s, A, y);
    }
    return z;
  }

  // a tightened bound with a multiplier of its sign holds through its row
  void undo_tightening(const psl_record& r, const HostCols& A, double* y) const {
    if (r.k < 0) return;
    double zj = reduced_cost_then(A, y, r.j);
    bool carries = (r.side == 0 && zj > 0.0) || (r.side == 1 && zj < 0.0);
    if (carries) y[r.k] = y[r.k] + zj / r.v[2];
  }

  // an active merged side of a leader belongs to the row that gave it
  void undo_merged_sides(const psl_record& r, double* y) const {
    int32_t leader = r.i;
    double yl = y[leader];
    int32_t giver = yl > 0.0 ? r.j : (yl < 0.0 ? r.k : -1);
    if (giver < 0 || giver == leader) return;
    auto it = row_lambda_.find(giver);
    y[giver] = yl / (it == row_lambda_.end() ? 0.0 : it->second);
    y[leader] = 0.0;
  }

  const psl_record* rec_;
  int64_t count_;
  bool needs_rows_ = false;
  std::vector<std::pair<int32_t, double>> fixed_;
  std::unordered_map<int64_t, ColumnGroup> groups_;  // keyed by the LEADER_BOUNDS record's position
  std::unordered_map<int32_t, double> row_lambda_;   // merged row -> lambda
  std::unordered_map<int32_t, int64_t> kept_by_;     // kept column -> its DOUBLETON_ROW record, not undone yet
  std::vector<std::pair<int32_t, double>> substituted_;  // FREE_SINGLETON row -> c_j / a_ij
};

}  // namespace

bool records_need_rows(const psl_record* rec, int64_t count) {
  for (int64_t t = 0; t < count; ++t)
    if (rec[t].type == T_FREE_SINGLETON) return true;
  return false;
}

psl_status postsolve_primal(const psl_record* rec, int64_t count, const int32_t* col_map_dev, int32_t n,
                            int32_t n_red, const double* x_red, double* x, const HostRows* rows, double inf_value,
                            std::string* err) {
  RecordStack st(rec, count);
  if (st.needs_rows() && !rows) {
    *err = "free-singleton records need the original rows, which this handle does not keep";
    return PSL_ERR_UNSUPPORTED;
  }
  std::vector<int32_t> kept(n_red);
  if (n_red && hipMemcpy(kept.data(), col_map_dev, n_red * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
    *err = "HIP error copying the column map";
    return PSL_ERR_DEVICE;
  }
  std::fill(x, x + n, 0.0);
  for (int32_t t = 0; t < n_red; ++t) x[kept[t]] = x_red[t];
  st.primal(x, rows, inf_value);
  return PSL_OK;
}

void postsolve_dual(const psl_record* rec, int64_t count, int32_t m, int32_t n, const std::vector<int32_t>& row_map,
                    const double* y_red, const HostCols& A, double* y, double* z) {
  std::fill(y, y + m, 0.0);
  for (size_t t = 0; t < row_map.size(); ++t) y[row_map[t]] = y_red[t];
  RecordStack st(rec, count);
  st.dual(A, y);
  for (int32_t j = 0; j < n; ++j) z[j] = RecordStack::reduced_cost(A, y, j);
}

}  // namespace psl
