// Host-side (FP64) setup of a cell type: mesh validation, triangle rest frames, bending
// stencils, lumped mass, assembly and factorisation of the constant system matrix L, its
// inverse, and the per-wave element schedules of the fused kernel.
//
// The method is the implicit-Euler step of the supplementary material (npFEM subsection):
// g(x) = 1/(2h^2) ||M^(1/2)(x - y)||^2 + sum_i E_i(x), minimised by the quasi-Newton
// iteration with a constant Hessian approximation. With projective-dynamics energies
// w/2 ||A x - p||^2 that approximation is L = M/h^2 + sum w A^T A, built here once per type.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <random>
#include <set>
#include <utility>

#include "npfem_internal.h"

namespace npfem {

namespace {

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }

// cot of the angle between u and v
inline double cot(V3 u, V3 v) { return dot(u, v) / norm(cross(u, v)); }

// ---- fused-kernel element schedules
//
// A schedule lists, round by round, the element each lane of a cell handles; the elements of
// one round share no vertex, so one wave accumulates their residuals into LDS without atomics.
// Each lane reads the positions of its element's vertices (one LDS access per vertex role and
// coordinate) and read-modify-writes the residuals at the same words. The LDS has 32 banks of
// 4 bytes; a wave64 access is served a half-wave at a time, each half taking as many cycles as
// its busiest bank has distinct words. Vertex v of a cell sits at word 3v + coordinate, so the
// bank of a role's access is fixed by v mod 32 (3 is odd). Two choices spread the accesses:
//   packing   which elements share a round: a residue class mod M should hold no more
//             vertices than there are roles (the arity), M = 32 when a cell fills a half-wave;
//   roles     which vertex of an element is read in which role: an edge colouring of the
//             bipartite multigraph (elements) x (residue classes) with arity colours, which
//             exists when every class has at most arity vertices (Koenig's theorem); a class
//             with more is split into sub-classes of at most arity vertices first.
// A few packings are tried and the one with the lowest modelled cost is kept (per round, the
// larger of its LDS cycles under the bank model and its VALU work per wave, plus part of the
// smaller).

struct Schedule {
  std::vector<std::vector<std::vector<int>>> rounds;  // [round][slot] -> vertices in role order
  std::vector<std::vector<int>> ids;                  // [round][slot] -> element
  double cost = 0.0;
};

// Greedy packing into rounds of at most `slots` vertex-disjoint elements. Elements touching
// the busiest vertices go first; each takes the fitting round with the fewest vertices beyond
// `cap` per residue class mod M (with `hard`, none beyond), then the least-filled one.
std::vector<std::vector<int>> pack_rounds(const std::vector<std::vector<int>>& elems, int n,
                                          int slots, int M, int cap, bool hard) {
  std::vector<int> deg(n, 0);
  for (auto& el : elems)
    for (int v : el) deg[v]++;
  std::vector<int> order(elems.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    int da = 0, db = 0;
    for (int v : elems[a]) da = std::max(da, deg[v]);
    for (int v : elems[b]) db = std::max(db, deg[v]);
    return da > db;
  });
  int max_deg = 0;
  for (int d : deg) max_deg = std::max(max_deg, d);
  const int lower = std::max<int>(max_deg, (int)((elems.size() + slots - 1) / slots));
  std::vector<std::vector<int>> rounds(lower);
  std::vector<std::vector<char>> used(lower, std::vector<char>(n, 0));
  std::vector<std::vector<int>> rc(lower, std::vector<int>(M, 0));
  for (int id : order) {
    int best = -1, best_over = 0;
    size_t best_fill = 0;
    for (int r = 0; r < (int)rounds.size(); ++r) {
      if (rounds[r].size() >= (size_t)slots) continue;
      bool ok = true;
      for (int v : elems[id])
        if (used[r][v]) { ok = false; break; }
      if (!ok) continue;
      int over = 0;
      for (size_t q = 0; q < elems[id].size(); ++q) {
        const int cls = elems[id][q] % M;
        int same = 0;   // earlier vertices of this element in the same class
        for (size_t p = 0; p < q; ++p) same += (elems[id][p] % M == cls);
        over += (rc[r][cls] + same >= cap);
      }
      if (hard && over > 0) continue;
      if (best < 0 || over < best_over || (over == best_over && rounds[r].size() < best_fill)) {
        best = r;
        best_over = over;
        best_fill = rounds[r].size();
      }
    }
    if (best < 0) {
      rounds.emplace_back();
      used.emplace_back(n, 0);
      rc.emplace_back(M, 0);
      best = (int)rounds.size() - 1;
    }
    rounds[best].push_back(id);
    for (int v : elems[id]) {
      used[best][v] = 1;
      rc[best][v % M]++;
    }
  }
  return rounds;
}

// Role assignment of one round: returns, per element, its vertices in role order such that
// within each role the vertices' residue classes mod M repeat as little as possible.
std::vector<std::vector<int>> assign_roles(const std::vector<std::vector<int>>& els, int M) {
  const int E = (int)els.size();
  if (E == 0) return {};
  const int arity = (int)els[0].size();
  // residue sub-classes: the c vertices of class r go round-robin to ceil(c / arity) nodes
  std::vector<int> cnt(M, 0);
  for (auto& el : els)
    for (int v : el) cnt[v % M]++;
  std::vector<int> first(M + 1, 0);
  for (int r = 0; r < M; ++r) first[r + 1] = first[r] + (cnt[r] + arity - 1) / arity;
  const int n_nodes = E + first[M];
  std::vector<int> seen(M, 0);
  struct Edge { int u, w, v; };
  std::vector<Edge> edges;
  for (int e = 0; e < E; ++e)
    for (int v : els[e]) {
      const int r = v % M, nsub = first[r + 1] - first[r];
      edges.push_back({e, E + first[r] + (seen[r]++ % nsub), v});
    }
  std::vector<int> at((size_t)n_nodes * arity, -1);   // node x colour -> edge
  std::vector<int> col(edges.size(), -1);
  auto free_colour = [&](int node) {
    for (int c = 0; c < arity; ++c)
      if (at[(size_t)node * arity + c] < 0) return c;
    return -1;
  };
  for (int id = 0; id < (int)edges.size(); ++id) {
    const int u = edges[id].u, w = edges[id].w;
    const int a = free_colour(u), b = free_colour(w);
    if (at[(size_t)w * arity + a] >= 0) {
      // swap colours a and b along the alternating path leaving w by its a-coloured edge;
      // afterwards a is free at w and still free at u (bipartite graph)
      std::vector<int> path;
      int node = w, c = a;
      while (at[(size_t)node * arity + c] >= 0) {
        const int pe = at[(size_t)node * arity + c];
        path.push_back(pe);
        node = (edges[pe].u == node) ? edges[pe].w : edges[pe].u;
        c = (c == a) ? b : a;
      }
      for (int pe : path) {
        at[(size_t)edges[pe].u * arity + col[pe]] = -1;
        at[(size_t)edges[pe].w * arity + col[pe]] = -1;
      }
      for (int pe : path) {
        col[pe] = (col[pe] == a) ? b : a;
        at[(size_t)edges[pe].u * arity + col[pe]] = pe;
        at[(size_t)edges[pe].w * arity + col[pe]] = pe;
      }
    }
    col[id] = a;
    at[(size_t)u * arity + a] = id;
    at[(size_t)w * arity + a] = id;
  }
  std::vector<std::vector<int>> out(E, std::vector<int>(arity, -1));
  for (int id = 0; id < (int)edges.size(); ++id) out[edges[id].u][col[id]] = edges[id].v;
  return out;
}

// Cycles of one wave64 LDS access to 4-byte words (negative: lane inactive).
int lds_access_cycles(const int* words) {
  int total = 0;
  for (int h = 0; h < 2; ++h) {
    int worst = 0;
    for (int i = 32 * h; i < 32 * h + 32; ++i) {
      if (words[i] < 0) continue;
      bool dup = false;   // count each distinct word once
      for (int j = 32 * h; j < i && !dup; ++j) dup = (words[j] == words[i]);
      if (dup) continue;
      int k = 0;
      for (int j = 32 * h; j < 32 * h + 32; ++j) {
        if (words[j] < 0 || (words[j] & 31) != (words[i] & 31)) continue;
        bool dj = false;
        for (int l = 32 * h; l < j && !dj; ++l) dj = (words[l] == words[j]);
        k += !dj;
      }
      worst = std::max(worst, k);
    }
    total += worst;
  }
  return total;
}

// Rows the empty slots of a round read, per role: the empty lanes of a role all read one row
// of their cell (the same word within a cell), the row of the first n with the fewest modelled
// LDS cycles for that role's access. Their writes are skipped, so any row of the cell serves.
// Returns the round's LDS cycles for one coordinate of every role.
int empty_rows(const std::vector<std::vector<int>>& rr, int arity, int gw, int slots,
               int cell_words, int n, std::vector<int>* rows) {
  int words[64], total = 0;
  if (rows) rows->assign(arity, 0);
  for (int q = 0; q < arity; ++q) {
    int best = -1, best_row = 0;
    const bool any_empty = (int)rr.size() < slots;
    for (int e = 0; e < (any_empty ? std::min(n, 96) : 1); ++e) {
      for (int lane = 0; lane < 64; ++lane) {
        const int cw = lane / slots, sl = lane % slots;
        words[lane] = cw >= gw ? -1 : cw * cell_words + 3 * (sl < (int)rr.size() ? rr[sl][q] : e);
      }
      const int c = lds_access_cycles(words);
      if (best < 0 || c < best) {
        best = c;
        best_row = e;
      }
    }
    total += best;
    if (rows) (*rows)[q] = best_row;
  }
  return total;
}

// Modelled cost of a schedule: per round, the larger of the LDS cycles of its accesses and its
// VALU instructions, plus a quarter of the smaller (the waves sharing a CU overlap the two only
// in part). Each role costs a position read, a residual read and a residual write per coordinate.
double schedule_cost(const std::vector<std::vector<std::vector<int>>>& rounds, int gw,
                     int slots, int cell_words, int n, double valu_per_round) {
  double cost = 0.0;
  for (auto& rr : rounds) {
    if (rr.empty()) continue;
    const int lds = 3 * 3 * empty_rows(rr, (int)rr[0].size(), gw, slots, cell_words, n, nullptr);
    cost += std::max((double)lds, valu_per_round) + 0.25 * std::min((double)lds, valu_per_round);
  }
  return cost;
}

int arity_of(const std::vector<std::vector<int>>& elems) {
  return elems.empty() ? 1 : (int)elems[0].size();
}

// Steps of the packing refinement per schedule (about 0.1 s for the 258-vertex RBC mesh).
constexpr long kRefineSteps = 1000000;

// Local search over the packing of one schedule. A step moves an element to another round
// that has a free slot, or swaps two elements of different rounds, keeping every round
// vertex-disjoint; the objective is the number of vertices beyond the arity per residue class
// mod M and round (with none beyond, the role assignment gives every role access distinct
// classes). Simulated annealing with a fixed seed and step count, so the result is the same on
// every run.
std::vector<std::vector<int>> refine_rounds(const std::vector<std::vector<int>>& elems, int n,
                                            int slots, int M, std::vector<std::vector<int>> rounds,
                                            long steps) {
  const int E = (int)elems.size(), R = (int)rounds.size();
  if (E == 0 || R < 2) return rounds;
  const int arity = (int)elems[0].size();
  std::vector<int> rnd(E), pos(E);
  std::vector<std::vector<int>> mem(R);
  std::vector<unsigned char> used((size_t)R * n, 0);
  std::vector<int> cnt((size_t)R * M, 0);
  long total = 0;
  auto add = [&](int e, int r, int sign) {
    for (int v : elems[e]) {
      int& c = cnt[(size_t)r * M + v % M];
      total -= std::max(0, c - arity);
      c += sign;
      total += std::max(0, c - arity);
      used[(size_t)r * n + v] = sign > 0;
    }
    if (sign > 0) {
      rnd[e] = r;
      pos[e] = (int)mem[r].size();
      mem[r].push_back(e);
    } else {
      const int last = mem[r].back();
      mem[r][pos[e]] = last;
      pos[last] = pos[e];
      mem[r].pop_back();
    }
  };
  for (int r = 0; r < R; ++r)
    for (int e : rounds[r]) add(e, r, 1);
  auto has = [&](int e, int v) {
    if (e < 0) return false;
    for (int x : elems[e])
      if (x == v) return true;
    return false;
  };
  std::mt19937_64 rng(0x6e70'6665'6d5fULL);
  const double t0 = 0.3;
  for (long it = 0; it < steps && total > 0; ++it) {
    const int e1 = (int)(rng() % (unsigned)E), r1 = rnd[e1];
    const int r2 = (int)(rng() % (unsigned)R);
    if (r2 == r1) continue;
    int e2 = -1;
    if ((int)mem[r2].size() >= slots || (!mem[r2].empty() && (rng() & 1))) e2 = mem[r2][rng() % mem[r2].size()];
    bool ok = true;
    for (int v : elems[e1])
      if (used[(size_t)r2 * n + v] && !has(e2, v)) ok = false;
    if (ok && e2 >= 0)
      for (int v : elems[e2])
        if (used[(size_t)r1 * n + v] && !has(e1, v)) ok = false;
    if (!ok) continue;
    const long before = total;
    add(e1, r1, -1);
    if (e2 >= 0) add(e2, r2, -1);
    add(e1, r2, 1);
    if (e2 >= 0) add(e2, r1, 1);
    const long d = total - before;
    const double temp = t0 * (1.0 - (double)it / (double)steps) + 0.02;
    if (d > 0 && (double)(rng() >> 11) * 0x1.0p-53 >= std::exp(-(double)d / temp)) {
      add(e1, r2, -1);
      if (e2 >= 0) add(e2, r1, -1);
      add(e1, r1, 1);
      if (e2 >= 0) add(e2, r2, 1);
    }
  }
  std::vector<std::vector<int>> out;   // rounds left empty by the moves are dropped
  for (int r = 0; r < R; ++r)
    if (!mem[r].empty()) {
      out.push_back(mem[r]);
      std::sort(out.back().begin(), out.back().end());
    }
  return out;
}

Schedule best_schedule_uncached(const std::vector<std::vector<int>>& elems, int n, int gw,
                                int slots, int cell_words, double valu_per_round) {
  Schedule best;
  bool have = false;
  const int m_role = std::min(slots, 32);
  auto make = [&](const std::vector<std::vector<int>>& packed) {
    Schedule s;
    for (auto& r : packed) {
      std::vector<std::vector<int>> els;
      for (int id : r) els.push_back(elems[id]);
      s.rounds.push_back(assign_roles(els, m_role));
      s.ids.push_back(r);
    }
    s.cost = schedule_cost(s.rounds, gw, slots, cell_words, n, valu_per_round);
    return s;
  };
  for (int M : {1, 2, 4, 8, 16, 32}) {
    if (M > m_role) break;
    for (int capf : {1, 2})
      for (int hard : {0, 1}) {
        if (M == 1 && (capf > 1 || hard)) continue;
        Schedule s = make(pack_rounds(elems, n, slots, M, M == 1 ? 1 << 30 : capf * arity_of(elems),
                                      hard != 0));
        if (!have || s.cost < best.cost ||
            (s.cost == best.cost && s.rounds.size() < best.rounds.size())) {
          best = std::move(s);
          have = true;
        }
      }
  }
  // the greedy packings leave residue classes crowded in most rounds: refine the best one
  if (have) {
    Schedule s = make(refine_rounds(elems, n, slots, m_role, best.ids, kRefineSteps));
    if (s.cost <= best.cost) best = std::move(s);
  }
  return best;
}

// Schedules depend only on the element lists and the layout, and their search takes a fraction
// of a second per schedule: the process keeps every schedule it built, keyed by all of its
// inputs, so types built again from the same mesh reuse it.
Schedule best_schedule(const std::vector<std::vector<int>>& elems, int n, int gw, int slots,
                       int cell_words, double valu_per_round) {
  static std::mutex mu;
  static std::map<std::vector<int64_t>, Schedule> cache;
  std::vector<int64_t> key{n, gw, slots, cell_words, (int64_t)std::llround(valu_per_round * 1024.0),
                           (int64_t)elems.size()};
  for (auto& el : elems) {
    key.push_back((int64_t)el.size());
    key.insert(key.end(), el.begin(), el.end());
  }
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  Schedule s = best_schedule_uncached(elems, n, gw, slots, cell_words, valu_per_round);
  std::lock_guard<std::mutex> lock(mu);
  cache.emplace(std::move(key), s);
  return s;
}

// D_m^-1 of the triangle (a, b, c): F = [x_b - x_a, x_c - x_a] D_m^-1 with D_m upper triangular
// in the frame whose first axis is b - a. Returns {gb0, gb1, gc0, gc1}.
std::array<double, 4> rest_frame(V3 a, V3 b, V3 c) {
  V3 e1 = sub(b, a), e2 = sub(c, a);
  double l1 = norm(e1);
  V3 t1 = scale(e1, 1.0 / l1);
  double d12 = dot(e2, t1);
  double l2 = norm(sub(e2, scale(t1, d12)));
  // D_m = [[l1, d12], [0, l2]],  D_m^-1 = [[1/l1, -d12/(l1 l2)], [0, 1/l2]]
  return {1.0 / l1, -d12 / (l1 * l2), 0.0, 1.0 / l2};
}

// Cholesky A = C C^T (lower, FP64, dense storage) of an SPD matrix whose nonzeros lie within
// bw of the diagonal; the factor keeps that band (zero fill outside it). False on a pivot
// that is not positive.
bool band_cholesky(const std::vector<double>& A, int n, int bw, std::vector<double>& C) {
  C.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    int k0 = std::max(0, j - bw);
    for (int k = k0; k < j; ++k) d -= C[(size_t)j * n + k] * C[(size_t)j * n + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    double cjj = std::sqrt(d);
    C[(size_t)j * n + j] = cjj;
    int i1 = std::min(n - 1, j + bw);
    for (int i = j + 1; i <= i1; ++i) {
      double s = A[(size_t)i * n + j];
      int kk = std::max(k0, i - bw);
      for (int k = kk; k < j; ++k) s -= C[(size_t)i * n + k] * C[(size_t)j * n + k];
      C[(size_t)i * n + j] = s / cjj;
    }
  }
  return true;
}

}  // namespace

npfem_status build_celltype(const npfem_mesh* mesh, const npfem_material* mat, double dt,
                            npfem_celltype* ct) {
  if (!mesh || !mat || !mesh->rest_xyz || !mesh->tri)
    return fail(NPFEM_E_INVALID, "null mesh or material");
  const int n = mesh->n_vertices, m = mesh->n_triangles;
  if (n < 4 || m < 4) return fail(NPFEM_E_MESH, "mesh needs >= 4 vertices and triangles");
  if (n > 65535) return fail(NPFEM_E_UNSUPPORTED, "meshes above 65535 vertices");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(NPFEM_E_INVALID, "dt must be > 0");
  if (!(mat->density > 0) || mat->shear_B < 0 || mat->area_C < 0 || mat->k_bend < 0 ||
      mat->k_vol < 0 || !(mat->strain_min > 0) || mat->strain_max < mat->strain_min ||
      !(mat->pbd_kappa >= 0.0 && mat->pbd_kappa <= 1.0) ||
      !(mat->v_max >= 0.0 && std::isfinite(mat->v_max)) ||
      !(mat->rayleigh_alpha >= 0.0 && std::isfinite(mat->rayleigh_alpha)) ||
      !(mat->rayleigh_beta >= 0.0 && std::isfinite(mat->rayleigh_beta)) ||
      (mat->membrane != NPFEM_MEMBRANE_PD && mat->membrane != NPFEM_MEMBRANE_SKALAK))
    return fail(NPFEM_E_INVALID, "material constants out of range");

  ct->n = n;
  ct->m = m;
  ct->h = dt;
  ct->w_s = mat->shear_B;
  ct->w_a = mat->area_C;
  ct->w_b = mat->k_bend;
  ct->w_v = mat->k_vol;
  ct->s_min = mat->strain_min;
  ct->s_max = mat->strain_max;
  ct->kappa = mat->pbd_kappa;
  ct->v_max = mat->v_max;
  ct->alpha = mat->rayleigh_alpha;
  ct->beta = mat->rayleigh_beta;
  ct->membrane = mat->membrane;
  if (ct->membrane == NPFEM_MEMBRANE_SKALAK && ct->beta > 0.0)
    return fail(NPFEM_E_UNSUPPORTED, "the Skalak membrane with Rayleigh beta damping");
  ct->X.assign(mesh->rest_xyz, mesh->rest_xyz + 3 * (size_t)n);
  ct->tri.assign(mesh->tri, mesh->tri + 3 * (size_t)m);
  for (double c : ct->X)
    if (!std::isfinite(c)) return fail(NPFEM_E_MESH, "non-finite rest coordinate");

  auto P = [&](int i) { return V3{ct->X[3 * i], ct->X[3 * i + 1], ct->X[3 * i + 2]}; };

  // ---- topology: closed, edge-manifold, consistently oriented, no unused vertex
  double ext = 0;
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) ext = std::max(ext, std::fabs(ct->X[3 * i + d] - ct->X[d]));
  std::map<std::pair<int, int>, int> opp;  // directed edge -> opposite vertex
  std::vector<int> used(n, 0);
  for (int t = 0; t < m; ++t) {
    int v[3] = {ct->tri[3 * t], ct->tri[3 * t + 1], ct->tri[3 * t + 2]};
    for (int r = 0; r < 3; ++r) {
      if (v[r] < 0 || v[r] >= n) return fail(NPFEM_E_MESH, "triangle index out of range");
      used[v[r]] = 1;
    }
    if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2])
      return fail(NPFEM_E_MESH, "triangle with a repeated vertex");
    double a2 = norm(cross(sub(P(v[1]), P(v[0])), sub(P(v[2]), P(v[0]))));
    if (!(a2 > 1e-12 * ext * ext)) return fail(NPFEM_E_MESH, "zero-area triangle");
    for (int r = 0; r < 3; ++r) {
      auto key = std::make_pair(v[r], v[(r + 1) % 3]);
      if (opp.count(key)) return fail(NPFEM_E_MESH, "directed edge used twice (non-manifold "
                                                    "or inconsistent orientation)");
      opp[key] = v[(r + 2) % 3];
    }
  }
  for (int i = 0; i < n; ++i)
    if (!used[i]) return fail(NPFEM_E_MESH, "vertex not used by any triangle");
  for (auto& kv : opp)
    if (!opp.count({kv.first.second, kv.first.first}))
      return fail(NPFEM_E_MESH, "open mesh: an edge has only one triangle");

  // ---- rest volume and area
  double V0 = 0, area0 = 0;
  for (int t = 0; t < m; ++t) {
    V3 a = P(ct->tri[3 * t]), b = P(ct->tri[3 * t + 1]), c = P(ct->tri[3 * t + 2]);
    V0 += dot(a, cross(b, c)) / 6.0;
    area0 += 0.5 * norm(cross(sub(b, a), sub(c, a)));
  }
  if (!(V0 > 0)) return fail(NPFEM_E_MESH, "rest volume <= 0 (triangles must be CCW from outside)");
  ct->V0 = V0;
  ct->area0 = area0;
  ct->mass = mat->density * V0 / n;

  // ---- triangle rest frames: F = [x_b - x_a, x_c - x_a] D_m^-1, D_m upper triangular
  ct->G.assign((size_t)m * 6, 0.0);
  ct->A.assign(m, 0.0);
  for (int t = 0; t < m; ++t) {
    V3 a = P(ct->tri[3 * t]), b = P(ct->tri[3 * t + 1]), c = P(ct->tri[3 * t + 2]);
    const auto fr = rest_frame(a, b, c);
    const double gb0 = fr[0], gb1 = fr[1], gc0 = fr[2], gc1 = fr[3];
    V3 e1 = sub(b, a), e2 = sub(c, a);
    double* g = &ct->G[6 * (size_t)t];
    g[2] = gb0; g[3] = gb1;
    g[4] = gc0; g[5] = gc1;
    g[0] = -gb0 - gc0; g[1] = -gb1 - gc1;
    ct->A[t] = 0.5 * norm(cross(e1, e2));
  }

  // ---- hinges: edge (i, j) with i < j in triangle (i, j, k), opposite l in (j, i, l)
  std::vector<std::array<int, 4>> hv;
  for (auto& kv : opp) {
    int i = kv.first.first, j = kv.first.second;
    if (i < j) hv.push_back({i, j, kv.second, opp[{j, i}]});
  }
  std::sort(hv.begin(), hv.end());
  const int e = (int)hv.size();
  ct->e = e;
  ct->hinge.resize(4 * (size_t)e);
  ct->coef.resize(4 * (size_t)e);
  ct->rest_norm.resize(e);
  for (int h = 0; h < e; ++h) {
    int i = hv[h][0], j = hv[h][1], k = hv[h][2], l = hv[h][3];
    V3 xi = P(i), xj = P(j), xk = P(k), xl = P(l);
    V3 e0 = sub(xj, xi), e1 = sub(xk, xi), e2 = sub(xl, xi), e3 = sub(xk, xj), e4 = sub(xl, xj);
    V3 me0 = scale(e0, -1.0);
    double c01 = cot(e0, e1), c02 = cot(e0, e2), c03 = cot(me0, e3), c04 = cot(me0, e4);
    double A0 = 0.5 * norm(cross(e0, e1)), A1 = 0.5 * norm(cross(e0, e2));
    double s = std::sqrt(3.0 / (A0 + A1));
    double a[4] = {s * (c03 + c04), s * (c01 + c02), -s * (c01 + c03), -s * (c02 + c04)};
    int idx[4] = {i, j, k, l};
    V3 u{0, 0, 0};
    for (int q = 0; q < 4; ++q) {
      ct->hinge[4 * h + q] = idx[q];
      ct->coef[4 * h + q] = a[q];
      V3 xq = P(idx[q]);
      u = {u.x + a[q] * xq.x, u.y + a[q] * xq.y, u.z + a[q] * xq.z};
    }
    ct->rest_norm[h] = norm(u);
  }

  // ---- system matrix L (FP64, dense; it is banded under the mesh's vertex order)
  std::vector<double>& L = ct->L;
  L.assign((size_t)n * n, 0.0);
  const double diag = ct->mass / (dt * dt) + ct->w_v;
  for (int i = 0; i < n; ++i) L[(size_t)i * n + i] = diag;
  for (int t = 0; t < m; ++t) {
    const double w = (ct->w_s + ct->w_a) * ct->A[t];
    const double* g = &ct->G[6 * (size_t)t];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        int vp = ct->tri[3 * t + p], vq = ct->tri[3 * t + q];
        L[(size_t)vp * n + vq] += w * (g[2 * p] * g[2 * q] + g[2 * p + 1] * g[2 * q + 1]);
      }
  }
  for (int h = 0; h < e; ++h)
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q < 4; ++q)
        L[(size_t)ct->hinge[4 * h + p] * n + ct->hinge[4 * h + q]] +=
            ct->w_b * ct->coef[4 * h + p] * ct->coef[4 * h + q];
  // ---- Rayleigh damping C = alpha M + beta K, K the element part of L assembled above:
  //      L = M~/h^2 + w_v I + K = ((1 + h alpha) m/h^2 + w_v) I + (1 + beta/h) K
  const bool rayleigh = ct->alpha != 0.0 || ct->beta != 0.0;
  std::vector<double> K;
  if (rayleigh) {
    K.assign((size_t)n * n, 0.0);   // the element part of L, summed from zero
    for (int t = 0; t < m; ++t) {
      const double w = (ct->w_s + ct->w_a) * ct->A[t];
      const double* g = &ct->G[6 * (size_t)t];
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
          int vp = ct->tri[3 * t + p], vq = ct->tri[3 * t + q];
          K[(size_t)vp * n + vq] += w * (g[2 * p] * g[2 * q] + g[2 * p + 1] * g[2 * q + 1]);
        }
    }
    for (int h = 0; h < e; ++h)
      for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q)
          K[(size_t)ct->hinge[4 * h + p] * n + ct->hinge[4 * h + q]] +=
              ct->w_b * ct->coef[4 * h + p] * ct->coef[4 * h + q];
    const double kb = 1.0 + ct->beta / dt;
    const double dd = (1.0 + dt * ct->alpha) * ct->mass / (dt * dt) + ct->w_v;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) L[(size_t)i * n + j] = kb * K[(size_t)i * n + j] + (i == j ? dd : 0.0);
  }
  int bw = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (L[(size_t)i * n + j] != 0.0) bw = std::max(bw, std::abs(i - j));
  ct->bw = bw;

  // ---- Cholesky L = C C^T (lower), FP64; zero fill outside the band is preserved
  std::vector<double>& C = ct->chol;
  if (!band_cholesky(L, n, bw, C)) return fail(NPFEM_E_NOT_SPD, "Cholesky pivot <= 0");
  ct->cband.assign((size_t)n * (bw + 1), 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k <= bw && k <= i; ++k) ct->cband[(size_t)i * (bw + 1) + k] = C[(size_t)i * n + i - k];
  // M~ = (1 + h alpha) m I + h beta K and the band of K, for the prediction's solve and the
  // gradient's damping term (beta > 0; with alpha alone M~ is diagonal)
  ct->mband.clear();
  ct->kband.clear();
  ct->pinv.clear();
  if (ct->beta > 0.0) {
    std::vector<double> Mt((size_t)n * n), Cm;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        Mt[(size_t)i * n + j] = dt * ct->beta * K[(size_t)i * n + j] +
                                (i == j ? (1.0 + dt * ct->alpha) * ct->mass : 0.0);
    if (!band_cholesky(Mt, n, bw, Cm)) return fail(NPFEM_E_NOT_SPD, "Cholesky pivot of M~ <= 0");
    // m M~^-1 column by column through M~'s factor (fused form)
    ct->pinv.assign((size_t)n * n, 0.0);
    std::vector<double> col(n);
    for (int c = 0; c < n; ++c) {
      std::fill(col.begin(), col.end(), 0.0);
      col[c] = ct->mass;
      for (int i = 0; i < n; ++i) {
        double s = col[i];
        for (int k = std::max(0, i - bw); k < i; ++k) s -= Cm[(size_t)i * n + k] * col[k];
        col[i] = s / Cm[(size_t)i * n + i];
      }
      for (int i = n - 1; i >= 0; --i) {
        double s = col[i];
        for (int k = i + 1; k <= std::min(n - 1, i + bw); ++k) s -= Cm[(size_t)k * n + i] * col[k];
        col[i] = s / Cm[(size_t)i * n + i];
      }
      for (int i = 0; i < n; ++i) ct->pinv[(size_t)i * n + c] = col[i];
    }
    ct->mband.assign((size_t)n * (bw + 1), 0.0);
    ct->kband.assign((size_t)n * (bw + 1), 0.0);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k <= bw && k <= i; ++k) {
        ct->mband[(size_t)i * (bw + 1) + k] = Cm[(size_t)i * n + i - k];
        ct->kband[(size_t)i * (bw + 1) + k] = K[(size_t)i * n + i - k];
      }
  }

  // ---- dense inverse: column by column through the factor (FP64)
  ct->Linv.assign((size_t)n * n, 0.0);
  std::vector<double> col(n);
  for (int c = 0; c < n; ++c) {
    std::fill(col.begin(), col.end(), 0.0);
    col[c] = 1.0;
    for (int i = 0; i < n; ++i) {
      double s = col[i];
      for (int k = std::max(0, i - bw); k < i; ++k) s -= C[(size_t)i * n + k] * col[k];
      col[i] = s / C[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = col[i];
      for (int k = i + 1; k <= std::min(n - 1, i + bw); ++k) s -= C[(size_t)k * n + i] * col[k];
      col[i] = s / C[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) ct->Linv[(size_t)i * n + c] = col[i];
  }

  // ---- vertex incidence (plain form gathers) and one-ring triangle pairs (fused form)
  ct->vt_off.assign(n + 1, 0);
  ct->vh_off.assign(n + 1, 0);
  for (int t = 0; t < m; ++t)
    for (int j = 0; j < 3; ++j) ct->vt_off[ct->tri[3 * t + j] + 1]++;
  for (int h = 0; h < e; ++h)
    for (int q = 0; q < 4; ++q) ct->vh_off[ct->hinge[4 * h + q] + 1]++;
  for (int i = 0; i < n; ++i) {
    ct->vt_off[i + 1] += ct->vt_off[i];
    ct->vh_off[i + 1] += ct->vh_off[i];
  }
  ct->vt_list.assign(ct->vt_off[n], 0);
  ct->vh_list.assign(ct->vh_off[n], 0);
  {
    std::vector<int> ft(ct->vt_off.begin(), ct->vt_off.end() - 1);
    std::vector<int> fh(ct->vh_off.begin(), ct->vh_off.end() - 1);
    for (int t = 0; t < m; ++t)
      for (int j = 0; j < 3; ++j) ct->vt_list[ft[ct->tri[3 * t + j]]++] = 3 * t + j;
    for (int h = 0; h < e; ++h)
      for (int q = 0; q < 4; ++q) ct->vh_list[fh[ct->hinge[4 * h + q]]++] = 4 * h + q;
  }
  ct->ring_info.assign(n, 0);
  ct->ring_pairs.assign(ct->vt_off[n], 0);
  int max_deg = 0;
  for (int i = 0; i < n; ++i) {
    int deg = ct->vt_off[i + 1] - ct->vt_off[i];
    max_deg = std::max(max_deg, deg);
    for (int s = 0; s < deg; ++s) {
      int code = ct->vt_list[ct->vt_off[i] + s];
      int t = code / 3, j = code % 3;
      int b = ct->tri[3 * t + (j + 1) % 3], c = ct->tri[3 * t + (j + 2) % 3];
      ct->ring_pairs[ct->vt_off[i] + s] = (uint32_t)b | ((uint32_t)c << 16);
    }
  }
  if (max_deg > 255) return fail(NPFEM_E_UNSUPPORTED, "vertex degree above 255");
  // each ring in cyclic order where the triangles chain (pair q + 1 starts where pair q ends,
  // c_q = b_{q+1}: the consecutive triangles around i share an edge), so that a walk around
  // the ring reads each neighbour once; a star of several cycles keeps them one after another
  for (int i = 0; i < n; ++i) {
    uint32_t* r = &ct->ring_pairs[ct->vt_off[i]];
    const int deg = ct->vt_off[i + 1] - ct->vt_off[i];
    for (int q = 0; q + 1 < deg; ++q) {
      const uint32_t c = r[q] >> 16;
      for (int u = q + 1; u < deg; ++u)
        if ((r[u] & 0xffffu) == c) {
          std::swap(r[q + 1], r[u]);
          break;
        }
    }
  }
  for (int i = 0; i < n; ++i)
    ct->ring_info[i] = ((uint32_t)ct->vt_off[i] << 8) | (uint32_t)(ct->vt_off[i + 1] - ct->vt_off[i]);
  // median-filter neighbour tables: the second vertex of each ring triangle (i, b, c) is every
  // neighbour once; short rings are padded evenly with -inf and +inf codes
  for (int keys : {8, 16}) {
    std::vector<uint16_t>& tab = keys == 8 ? ct->ring_nb8 : ct->ring_nb16;
    tab.assign((size_t)n * keys, kPadPos);
    for (int i = 0; i < n; ++i) {
      const int deg = ct->vt_off[i + 1] - ct->vt_off[i];
      uint16_t* row = &tab[(size_t)i * keys];
      row[0] = (uint16_t)deg;
      if (deg + 1 > keys) continue;
      const int neg = (keys - 1 - deg) / 2;
      for (int q = 0; q < keys - 1; ++q)
        row[1 + q] = q < deg ? (uint16_t)((ct->ring_pairs[ct->vt_off[i] + q] & 0xffffu) + kNbBias)
                             : (q - deg < neg ? kPadNeg : kPadPos);
    }
  }

  // ---- fused-form layout and element schedules
  // k rows per cell: whole MFMA k steps of 4 rows, at least one chunk of kMfmaChunk steps
  // (the global step's loads read whole chunks). A cell block of X or R holds 3 npad words
  // [vertex][xyz] plus pad words up to a stride cs = 3 (mod 16): with the k-row order of the
  // global step (in each chunk of 32 rows, the two lane groups of a half-wave read rows 16
  // apart) every 16-column B tile then reads 32 distinct LDS banks per half-wave, for any
  // number of cells in the group (32 banks of 4 bytes, served a half-wave at a time).
  const int npad = std::max((n + 3) / 4 * 4, 4 * kMfmaChunk);
  ct->npad = npad;
  ct->cs = 3 * npad + (((3 - 3 * npad) % 16) + 16) % 16;
  // X blocks in the first half of the LDS budget; R blocks, plus the per-cell damping data
  // when the type is damped, in the second (FP32)
  const bool skalak = ct->membrane == NPFEM_MEMBRANE_SKALAK;
  const int per_cell = ct->cs * 4 + (ct->kappa > 0.0 ? kDampWords * 4 : 0);
  std::vector<int> feasible;
  for (int cand : {16, 8, 4, 2, 1}) {
    if (kFusedWaves * cand * per_cell > 4 * kFusedRWords) continue;
    if (skalak && cand > kSkalakMaxGw) continue;
    if ((cand * n + 63) / 64 > kMaxItems) continue;
    if (kFusedWaves * cand > kMaxGroupCells) continue;
    // every wave's share of the global step's output tiles, for every group size, must form
    // at most kMaxTilesPerWave / 2 items (the kernel holds two tiles per item)
    bool fits = true;
    const int rt_n = (n + 15) / 16;
    for (int count = 1; count <= kFusedWaves * cand && fits; ++count) {
      const int ct_n = (3 * count + 15) / 16, units = rt_n * ct_n;
      for (int w = 0; w < kFusedWaves && fits; ++w)
        fits = mfma_share_items(ct_n, units * w / kFusedWaves, units * (w + 1) / kFusedWaves) <=
               kMaxTilesPerWave / 2;
    }
    if (fits) feasible.push_back(cand);
  }
  ct->fused_ok = !feasible.empty();
  if (!ct->fused_ok) {
    ct->fused_reason = "mesh too large for the fused kernel's LDS layout (n <= 576)";
    return NPFEM_OK;
  }
  if (skalak && ct->beta > 0.0) {
    ct->fused_ok = false;
    ct->fused_reason = "the Skalak membrane with Rayleigh beta runs in neither form";
    return NPFEM_OK;
  }

  std::vector<std::vector<int>> tel(m), hel(e);
  for (int t = 0; t < m; ++t) tel[t] = {ct->tri[3 * t], ct->tri[3 * t + 1], ct->tri[3 * t + 2]};
  for (int h = 0; h < e; ++h)
    hel[h] = {ct->hinge[4 * h], ct->hinge[4 * h + 1], ct->hinge[4 * h + 2], ct->hinge[4 * h + 3]};
  // approximate VALU instructions per wave of one triangle / hinge round of the fused
  // kernel (its gfx950 code), weighed against the rounds' modelled LDS cycles
  const double kTriRoundValu = 270.0, kHingeRoundValu = 81.0;
  for (int gw : feasible) {
    FusedLayout lay;
    lay.gw = gw;
    lay.slots = 64 / gw;
    const Schedule tr = best_schedule(tel, n, gw, lay.slots, ct->cs, kTriRoundValu);
    const Schedule hr = best_schedule(hel, n, gw, lay.slots, ct->cs, kHingeRoundValu);
    lay.tri_rounds = (int)tr.rounds.size();
    lay.hinge_rounds = (int)hr.rounds.size();
    // empty slots (orient 0 and area 0, or rest < 0: their writes are skipped) read the rows
    // that empty_rows chose for their round and role
    TriRec empty_tri{};
    lay.tri_sched.assign((size_t)lay.tri_rounds * lay.slots, empty_tri);
    HingeRec empty_hinge{};
    empty_hinge.rest = -1.0f;
    lay.hinge_sched.assign((size_t)lay.hinge_rounds * lay.slots, empty_hinge);
    std::vector<int> er;
    for (int r = 0; r < lay.tri_rounds; ++r) {
      empty_rows(tr.rounds[r], 3, gw, lay.slots, ct->cs, n, &er);
      for (size_t s = tr.rounds[r].size(); s < (size_t)lay.slots; ++s) {
        TriRec& rec = lay.tri_sched[(size_t)r * lay.slots + s];
        rec.a = 12u * (uint32_t)er[0];
        rec.b = 12u * (uint32_t)er[1];
        rec.c = 12u * (uint32_t)er[2];
      }
    }
    for (int r = 0; r < lay.hinge_rounds; ++r) {
      empty_rows(hr.rounds[r], 4, gw, lay.slots, ct->cs, n, &er);
      for (size_t s = hr.rounds[r].size(); s < (size_t)lay.slots; ++s) {
        HingeRec& rec = lay.hinge_sched[(size_t)r * lay.slots + s];
        rec.i = 12u * (uint32_t)er[0];
        rec.j = 12u * (uint32_t)er[1];
        rec.k = 12u * (uint32_t)er[2];
        rec.l = 12u * (uint32_t)er[3];
      }
    }
    for (int r = 0; r < lay.tri_rounds; ++r)
      for (size_t s = 0; s < tr.rounds[r].size(); ++s) {
        // roles (a, b, c) in the order the schedule chose; the rest frame follows it
        const auto& v = tr.rounds[r][s];
        const int t = tr.ids[r][s];
        const auto fr = rest_frame(P(v[0]), P(v[1]), P(v[2]));
        TriRec rec;
        rec.a = 12u * (uint32_t)v[0];
        rec.b = 12u * (uint32_t)v[1];
        rec.c = 12u * (uint32_t)v[2];
        rec.gb0 = (float)fr[0]; rec.gb1 = (float)fr[1];
        rec.gc1 = (float)fr[3];   // fr[2] = g_c0 = 0 in this rest frame
        rec.area = (float)ct->A[t];
        // the roles may reverse the triangle's orientation, which the volume terms see
        int k0 = 0;
        while (ct->tri[3 * t + k0] != v[0]) ++k0;
        rec.orient = (ct->tri[3 * t + (k0 + 1) % 3] == v[1]) ? 1.0f : -1.0f;
        lay.tri_sched[(size_t)r * lay.slots + s] = rec;
      }
    for (int r = 0; r < lay.hinge_rounds; ++r)
      for (size_t s = 0; s < hr.rounds[r].size(); ++s) {
        // any vertex may lead the difference form: the stencil's coefficients sum to zero
        const auto& v = hr.rounds[r][s];
        const int h = hr.ids[r][s];
        double a[4];
        for (int q = 0; q < 4; ++q)
          for (int p = 0; p < 4; ++p)
            if (ct->hinge[4 * h + p] == v[q]) a[q] = ct->coef[4 * h + p];
        HingeRec rec;
        rec.i = 12u * (uint32_t)v[0];
        rec.j = 12u * (uint32_t)v[1];
        rec.k = 12u * (uint32_t)v[2];
        rec.l = 12u * (uint32_t)v[3];
        rec.a1 = (float)a[1]; rec.a2 = (float)a[2]; rec.a3 = (float)a[3];
        rec.rest = (float)ct->rest_norm[h];
        lay.hinge_sched[(size_t)r * lay.slots + s] = rec;
      }
    // ring gather of the fused Skalak energy: the wave's gw n vertices by ring length (longest
    // first, then cell and vertex), 64 to a slot, so that the long rings of a mesh (the poles
    // of a UV sphere) share one slot and the wave walks each slot's longest ring once
    {
      std::vector<std::pair<int, int>> vs;   // (-ring length, code)
      for (int cw = 0; cw < gw; ++cw)
        for (int v = 0; v < n; ++v) vs.push_back({-(ct->vt_off[v + 1] - ct->vt_off[v]), (cw << 12) | v});
      std::stable_sort(vs.begin(), vs.end(),
                       [](const std::pair<int, int>& x, const std::pair<int, int>& y) { return x.first < y.first; });
      lay.gather_slots = (int)((vs.size() + 63) / 64);
      lay.gather_sched.assign((size_t)kMaxItems * 64, kGatherEmpty);
      for (size_t k = 0; k < vs.size(); ++k) lay.gather_sched[k] = (uint16_t)vs[k].second;
    }
    ct->layouts.push_back(std::move(lay));
  }
  ct->gw = ct->layouts[0].gw;
  ct->slots = ct->layouts[0].slots;
  ct->tri_rounds = ct->layouts[0].tri_rounds;
  ct->hinge_rounds = ct->layouts[0].hinge_rounds;
  return NPFEM_OK;
}

}  // namespace npfem
