// Host-side checks and exact arithmetic of the C ABI (host.cpp); no HIP.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mslm.h"

namespace mslm {

// One solve's reduced parameters: gamma = p/q, omega = a/b.
struct SolveSpec {
  int64_t p = 1, q = 1, a = 1, b = 1;
  int32_t max_levels = 32, max_iterations = 2, max_sweeps = 32;
  int32_t null_model = MSLM_NULL_MULTISLICE;
  uint64_t seed = 0;
  // per-slice resolutions gamma^(s) = gn[s]/gd[s] (reduced); empty: p/q in every slice
  std::vector<int64_t> gn, gd;
  // the start partition of the first iteration [T*N]; empty: singletons
  std::vector<int32_t> init;
  // The constants of the exact gains.  With Q = lcm_s gd_s, P_s = gn_s * Q / gd_s and
  // C = lcm_s P_s, slice s's null term gamma^(s) k y / S_s equals (C/Q) k y / (S_s * smul_s)
  // with smul_s = C / P_s, so the kernels' values qe*S'*W - pe*b*k*y (pe = C, qe = Q,
  // S' = S_s * smul_s) order targets as Eq. 6's gains do.  One resolution: pe = p, qe = q and
  // smul empty (every multiplier 1).
  int64_t pe = 1, qe = 1;
  std::vector<int64_t> smul;
};

mslm_status api_fail(mslm_status s, const std::string &m);   // sets the error text
void api_clear_error();
const char *api_error_text();
mslm_status api_check_shape(const mslm_graph_desc *d);
mslm_status api_check_desc(const mslm_graph_desc *d);        // shape, then host edge lists
mslm_status api_check_fraction(int64_t num, int64_t den, const char *what);
int64_t api_gcd(int64_t a, int64_t b);
// Validates and reduces a solve's parameters for a graph of N nodes and T slices (on, od: the
// graph's default coupling), copying the per-slice resolutions and the start partition.
mslm_status api_make_spec(const mslm_params *p, int64_t on, int64_t od, int32_t N, int32_t T,
                          SolveSpec &sp);
// The kernels' denominator of slice s (2m_s, or 1 under the CPM, times the slice's multiplier)
// and the int64 head-room of that slice's gains: S' < 2^31, qe*S'*(b*max(2m_s,1) + 2a) < 2^62
// and pe*b*K^2 < 2^62 with K = max(2m_s, 1), or N under the CPM.  False with the error text
// set when a bound fails.
// crow_s bounds a copy's coupling weight in slice s in units of omega (sum over r of c_sr).
bool api_slice_denominator(const SolveSpec &sp, int s, int64_t two_m, int64_t N, int64_t crow_s,
                           int64_t &Sdev);
// The coupling matrix of a graph description (c_sr, row-major T*T; ordinal when NULL), the
// per-slice row sums, the number of coupled slice pairs s < r, and on host edge lists the
// coupling total (sum of c_sr over ordered coupled copy pairs, present copies only when the
// description asks for that).
std::vector<int32_t> api_coupling_matrix(const mslm_graph_desc *d);
std::vector<int64_t> api_coupling_rows(const std::vector<int32_t> &cm, int T);
int64_t api_coupled_pairs(const std::vector<int32_t> &cm, int T);
int64_t api_coupling_total_host(const mslm_graph_desc *d);
// The head-room preconditions of a solve on host edge lists (2m_s < 2^31 per slice, then
// api_slice_denominator per slice, or the global null model's).
mslm_status api_check_headroom(const mslm_graph_desc *d, const SolveSpec &sp);
// Q of any objective of a solve from its 3T+1 components (the spec's null model and
// resolutions) as a reduced decimal fraction and the nearest double.
// ctot: the graph's coupling total (2mu = sum 2m_s + omega ctot).
mslm_status api_q_exact_spec(const int64_t *c, int T, int N, int64_t ctot, const SolveSpec &sp,
                             std::string &num, std::string &den, double &qd);
// Q of Eq. 6 (cpm = false) or of the multislice CPM from the components with a resolution
// gn[s]/gd[s] per slice.
mslm_status api_q_exact_slices(const int64_t *c, int T, int N, int64_t ctot, const int64_t *gn,
                               const int64_t *gd, bool cpm, int64_t oa, int64_t ob,
                               std::string &num, std::string &den, double &qd);
// Q of Eq. 6 from its 3T+1 components as a reduced decimal fraction and the nearest double.
mslm_status api_q_exact(const int64_t *c, int T, int N, int64_t gp, int64_t gq, int64_t oa,
                        int64_t ob, std::string &num, std::string &den, double &qd);
// Result-invariant execution choices (mslm_tuning)
struct Tuning {
  int graphs = 0;
  int64_t latency_units = 1024, split_group_units = 16384, copy_moves = 1024;
  int lat_parts_max = 16;
  int64_t batch_units = 24ll << 20;
};
mslm_status api_tuning_from(const mslm_tuning *t, Tuning &out);
void api_tuning_to(const Tuning &t, mslm_tuning *out);

// Q_G of the global null model from its components (the same layout, SS' in slot T).
mslm_status api_q_exact_global(const int64_t *c, int T, int N, int64_t ctot, int64_t gp, int64_t gq, int64_t oa,
                               int64_t ob, std::string &num, std::string &den, double &qd);
// The head-room preconditions of the global null model for one graph (2mu' as defined in the
// header); false with the error text set when they fail.
bool api_global_headroom(int64_t two_mu, const SolveSpec &sp);
// 2mu' = b * sum_s 2m_s + a * ctot, saturated at 2^62
int64_t global_two_mu(int64_t sum_two_m, int64_t ctot, const SolveSpec &sp);
// Device bytes of one solve's work buffers on a resident graph (upper estimate), and of a
// graph plus one solve.
size_t solve_scratch_estimate(int64_t n, int64_t nnz);
size_t footprint_estimate(const mslm_graph_desc *d);

}  // namespace mslm
