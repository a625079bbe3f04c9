// Host-side mesh topology and dual-cell tables (see geometry.hpp).
#include "geometry.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <thread>
#include <unordered_map>

namespace pmchwt {

namespace {
inline uint64_t key2(int32_t a, int32_t b) { return (uint64_t(uint32_t(a)) << 32) | uint32_t(b); }
}  // namespace

bool build_topology(const double* v, int nv, const int32_t* t, int F, Topo& T, std::string& err) {
  if (nv < 4 || F < 4) {
    err = "mesh too small to be closed";
    return false;
  }
  T.nv = nv;
  T.F = F;
  T.v.assign(v, v + 3 * size_t(nv));
  T.t.assign(t, t + 3 * size_t(F));
  for (int i = 0; i < 3 * F; ++i)
    if (t[i] < 0 || t[i] >= nv) {
      err = "triangle index out of range";
      return false;
    }
  // directed half edges -> (triangle, local index of the opposite vertex)
  std::unordered_map<uint64_t, int32_t> half;
  half.reserve(size_t(3) * F * 2);
  for (int f = 0; f < F; ++f)
    for (int a = 0; a < 3; ++a) {
      int32_t u = t[3 * f + (a + 1) % 3], w = t[3 * f + (a + 2) % 3];
      if (u == w) {
        err = "degenerate triangle (repeated vertex)";
        return false;
      }
      if (!half.emplace(key2(u, w), 3 * f + a).second) {
        err = "non-manifold or inconsistently oriented mesh";
        return false;
      }
    }
  std::vector<uint64_t> keys;
  keys.reserve(half.size() / 2);
  for (auto& kv : half) {
    int32_t u = int32_t(kv.first >> 32), w = int32_t(kv.first & 0xffffffffu);
    if (u < w) keys.push_back(kv.first);
  }
  std::sort(keys.begin(), keys.end());
  T.E = int(keys.size());
  if (size_t(2) * T.E != size_t(3) * F) {
    err = "open mesh: some edge has a single triangle";
    return false;
  }
  T.edges.resize(2 * size_t(T.E));
  T.tplus.resize(T.E);
  T.tminus.resize(T.E);
  T.t2e.assign(3 * size_t(F), -1);
  T.sgn.assign(3 * size_t(F), 0);
  for (int e = 0; e < T.E; ++e) {
    int32_t lo = int32_t(keys[e] >> 32), hi = int32_t(keys[e] & 0xffffffffu);
    auto p = half.find(key2(lo, hi));
    auto m = half.find(key2(hi, lo));
    if (m == half.end()) {
      err = "open mesh: edge traversed in one direction only";
      return false;
    }
    T.edges[2 * e] = lo;
    T.edges[2 * e + 1] = hi;
    T.tplus[e] = p->second / 3;
    T.tminus[e] = m->second / 3;
    T.t2e[p->second] = e;
    T.sgn[p->second] = 1;
    T.t2e[m->second] = e;
    T.sgn[m->second] = -1;
  }
  T.area.resize(F);
  T.normal.resize(3 * size_t(F));
  for (int f = 0; f < F; ++f) {
    const double* A = &v[3 * t[3 * f]];
    const double* B = &v[3 * t[3 * f + 1]];
    const double* C = &v[3 * t[3 * f + 2]];
    double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double w[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    double c[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    double n = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    if (!(n > 0.0)) {
      err = "degenerate triangle (zero area)";
      return false;
    }
    T.area[f] = 0.5 * n;
    for (int d = 0; d < 3; ++d) T.normal[3 * f + d] = c[d] / n;
  }
  return true;
}

bool build_dual(const Topo& T, DualCells& D, std::string& err) {
  const int nv = T.nv, E = T.E, F = T.F;
  D.nbv = nv + E + F;
  D.bv.resize(3 * size_t(D.nbv));
  for (int i = 0; i < 3 * nv; ++i) D.bv[i] = T.v[i];
  for (int e = 0; e < E; ++e)
    for (int d = 0; d < 3; ++d)
      D.bv[3 * (nv + e) + d] = 0.5 * (T.v[3 * T.edges[2 * e] + d] + T.v[3 * T.edges[2 * e + 1] + d]);
  for (int f = 0; f < F; ++f)
    for (int d = 0; d < 3; ++d)
      D.bv[3 * (nv + E + f) + d] =
          (T.v[3 * T.t[3 * f] + d] + T.v[3 * T.t[3 * f + 1] + d] + T.v[3 * T.t[3 * f + 2] + d]) / 3.0;
  // children and the primal vertex whose dual cell contains them
  D.child_vid.resize(18 * size_t(F));
  std::vector<int32_t> cellv(6 * size_t(F));
  for (int f = 0; f < F; ++f) {
    int32_t a = T.t[3 * f], b = T.t[3 * f + 1], c = T.t[3 * f + 2];
    int32_t mab = nv + T.t2e[3 * f + 2], mbc = nv + T.t2e[3 * f + 0], mca = nv + T.t2e[3 * f + 1];
    int32_t g = nv + E + f;
    int32_t ch[6][3] = {{a, mab, g}, {mab, b, g}, {b, mbc, g}, {mbc, c, g}, {c, mca, g}, {mca, a, g}};
    int32_t cv[6] = {a, b, b, c, c, a};
    for (int j = 0; j < 6; ++j) {
      for (int d = 0; d < 3; ++d) D.child_vid[18 * size_t(f) + 3 * j + d] = ch[j][d];
      cellv[6 * size_t(f) + j] = cv[j];
    }
  }
  // children per cell
  std::vector<std::vector<int32_t>> cells(nv);
  for (int c = 0; c < 6 * F; ++c) cells[cellv[c]].push_back(c);
  // incident edges per vertex
  std::vector<std::vector<int32_t>> inc(nv);
  for (int e = 0; e < E; ++e) {
    inc[T.edges[2 * e]].push_back(e);
    inc[T.edges[2 * e + 1]].push_back(e);
  }
  D.cell_ptr.assign(nv + 1, 0);
  D.inc_ptr.assign(nv + 1, 0);
  D.coef_ptr.assign(nv + 1, 0);
  D.max_valence = 0;
  for (int v = 0; v < nv; ++v) {
    int n2 = int(cells[v].size());
    if (n2 < 6 || (n2 & 1) || int(inc[v].size()) * 2 != n2) {
      err = "vertex star is not a disc";
      return false;
    }
    D.max_valence = std::max(D.max_valence, n2 / 2);
    D.cell_ptr[v + 1] = D.cell_ptr[v] + n2;
    D.inc_ptr[v + 1] = D.inc_ptr[v] + n2 / 2;
    D.coef_ptr[v + 1] = D.coef_ptr[v] + int64_t(n2 / 2) * n2;
  }
  D.ring.resize(D.cell_ptr[nv]);
  D.inc_edges.resize(D.inc_ptr[nv]);
  D.coef.assign(4 * size_t(D.coef_ptr[nv]), 0.0);
  D.bbox.resize(6 * size_t(E));

  auto child_pts = [&](int32_t c, double P[3][3]) {
    for (int k = 0; k < 3; ++k)
      for (int d = 0; d < 3; ++d) P[k][d] = D.bv[3 * size_t(D.child_vid[3 * size_t(c) + k]) + d];
  };
  // the two radial edges of a child in cell v are (v, m) and (v, g); a child
  // is identified by its "other endpoints" (m, g).  The boundary edge (m, g)
  // is opposite v.
  // one dual cell (independent of the others: disjoint output ranges)
  auto cell = [&](int v, std::string& err) -> bool {
    const std::vector<int32_t>& cl = cells[v];
    int n2 = int(cl.size()), N = n2 / 2;
    std::map<int32_t, std::vector<int32_t>> by_key;  // other endpoint -> children
    std::vector<int32_t> mkey(n2), gkey(n2);
    for (int i = 0; i < n2; ++i) {
      int32_t m = -1, g = -1;
      for (int k = 0; k < 3; ++k) {
        int32_t id = D.child_vid[3 * size_t(cl[i]) + k];
        if (id == v) continue;
        if (id >= nv + E) g = id; else m = id;
      }
      mkey[i] = m;
      gkey[i] = g;
      by_key[m].push_back(i);
      by_key[g].push_back(i);
    }
    // walk the ring: alternate crossing the (v,g) and (v,m) radial edges
    std::vector<int> order;
    order.reserve(n2);
    int cur = 0;
    bool via_g = true;
    std::vector<char> seen(n2, 0);
    for (int s = 0; s < n2; ++s) {
      order.push_back(cur);
      seen[cur] = 1;
      int32_t key = via_g ? gkey[cur] : mkey[cur];
      const auto& nb = by_key[key];
      if (nb.size() != 2) {
        err = "barycentric ring broken";
        return false;
      }
      int nxt = nb[0] == cur ? nb[1] : nb[0];
      if (s + 1 < n2 && seen[nxt]) {
        err = "barycentric ring does not close";
        return false;
      }
      cur = nxt;
      via_g = !via_g;
    }
    for (int i = 0; i < n2; ++i) D.ring[D.cell_ptr[v] + i] = cl[order[i]];
    // incident edges: the ones whose midpoint key appears in the cell
    for (int s = 0; s < N; ++s) D.inc_edges[D.inc_ptr[v] + s] = inc[v][s];
    // per incident edge: rotate the ring so that t_1, t_2N share half edge (v, m_e)
    std::vector<int32_t> rm(n2), rg(n2);
    for (int i = 0; i < n2; ++i) {
      rm[i] = mkey[order[i]];
      rg[i] = gkey[order[i]];
    }
    for (int s = 0; s < N; ++s) {
      int32_t e = inc[v][s];
      int32_t me = nv + e;
      double sigma = (T.edges[2 * e] == v) ? 1.0 : -1.0;
      // find r with ring[r] and ring[r-1] both carrying m_e and adjacent via it
      int r = -1;
      for (int i = 0; i < n2; ++i) {
        int ip = (i + n2 - 1) % n2;
        if (rm[i] == me && rm[ip] == me) {
          r = i;
          break;
        }
      }
      if (r < 0) {
        err = "edge midpoint not found in its vertex ring";
        return false;
      }
      for (int k = 1; k <= n2; ++k) {
        int pos = (r + k - 1) % n2;         // ring position of t_k
        int32_t child = D.ring[D.cell_ptr[v] + pos];
        int ci = order[pos];
        // fluxes: toward t_{k+1} and toward t_{k-1}, both radial
        double f_next = (k < n2) ? sigma * double(k - N) / (2.0 * N) : 0.0;
        double f_prev = (k > 1) ? -sigma * double(k - 1 - N) / (2.0 * N) : 0.0;
        double f_exit = (k == 1 || k == n2) ? 0.5 * sigma : 0.0;
        // which radial edge leads to t_{k+1}?  ring alternates g/m crossings
        int32_t next_key = (k < n2) ? ((rg[pos] == rg[(pos + 1) % n2]) ? rg[pos] : rm[pos]) : -1;
        int32_t prev_key = (k > 1) ? ((rg[pos] == rg[(pos + n2 - 1) % n2]) ? rg[pos] : rm[pos]) : -1;
        double P[3][3];
        child_pts(child, P);
        double A2;
        {
          double u[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
          double w[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
          double c[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
          A2 = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);  // 2 * area
        }
        // flux through the edge opposite each local vertex
        double phi[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
          int32_t id = D.child_vid[3 * size_t(child) + a];
          if (id == v) {
            phi[a] = f_exit;                           // opposite v: boundary edge (m, g)
          } else {
            // opposite id: the radial edge (v, other) with other != id
            int32_t other = (id == mkey[ci]) ? gkey[ci] : mkey[ci];
            double f = 0.0;
            if (other == next_key) f += f_next;
            if (other == prev_key) f += f_prev;
            phi[a] = f;
          }
        }
        double alpha = (phi[0] + phi[1] + phi[2]) / A2;
        double w[3];
        for (int d = 0; d < 3; ++d) w[d] = (phi[0] * P[0][d] + phi[1] * P[1][d] + phi[2] * P[2][d]) / A2;
        size_t rec = size_t(D.coef_ptr[v]) + size_t(s) * n2 + pos;
        D.coef[4 * rec + 0] = alpha;
        D.coef[4 * rec + 1] = w[0];
        D.coef[4 * rec + 2] = w[1];
        D.coef[4 * rec + 3] = w[2];
      }
    }
    return true;
  };
  // cells in parallel ranges on large meshes
  const int nthreads = nv >= 2048 ? int(std::max(1u, std::min(8u, std::thread::hardware_concurrency()))) : 1;
  std::vector<std::string> errs(nthreads);
  std::vector<char> ok(nthreads, 1);
  auto range = [&](int w) {
    for (int v = int(int64_t(nv) * w / nthreads); v < int(int64_t(nv) * (w + 1) / nthreads); ++v)
      if (!cell(v, errs[w])) {
        ok[w] = 0;
        return;
      }
  };
  if (nthreads == 1) {
    range(0);
  } else {
    std::vector<std::thread> pool;
    for (int w = 0; w < nthreads; ++w) pool.emplace_back(range, w);
    for (auto& t : pool) t.join();
  }
  for (int w = 0; w < nthreads; ++w)
    if (!ok[w]) {
      err = errs[w];
      return false;
    }
  // bounding boxes of BC supports: both dual cells
  for (int e = 0; e < E; ++e) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int end = 0; end < 2; ++end) {
      int v = T.edges[2 * e + end];
      for (int i = D.cell_ptr[v]; i < D.cell_ptr[v + 1]; ++i)
        for (int k = 0; k < 3; ++k) {
          int32_t id = D.child_vid[3 * size_t(D.ring[i]) + k];
          for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], D.bv[3 * size_t(id) + d]);
            hi[d] = std::max(hi[d], D.bv[3 * size_t(id) + d]);
          }
        }
    }
    for (int d = 0; d < 3; ++d) {
      D.bbox[6 * size_t(e) + d] = lo[d];
      D.bbox[6 * size_t(e) + 3 + d] = hi[d];
    }
  }
  return true;
}

}  // namespace pmchwt
