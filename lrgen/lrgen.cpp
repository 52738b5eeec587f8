// Seeded synthesis of trivariate LR-spline volumes by local refinement of an
// open tensor-product mesh on [0,1]^3 (input generation only; no rendering,
// evaluation or extraction arithmetic lives here).
//
// An LR-spline (Eq. 2, Sec. 3.1) is a sum c_i * gamma_i * N_i over LR
// B-splines N_i, each a tensor B-spline on its own local knot vectors of
// p_d + 2 knots per axis.  It is produced from a tensor mesh by inserting
// axis-parallel mesh rectangles and then splitting every LR B-spline whose
// support is traversed by a mesh rectangle it does not carry, until all are of
// minimal support (Sec. 3.1).  One refinement here inserts the rectangle
// {x_a = m} x (support of N* on the two other axes), where m halves the
// element that holds a seed point along its longest side and N* is the
// smallest B-spline whose support covers that element.
//
// Splitting uses 1-D knot insertion of one knot into one B-spline:
//   B[u_0..u_{p+1}] = a1 * B[first p+2 knots of u+{v}] + a2 * B[last p+2 knots]
//   a1 = (v - u_0) / (u_p - u_0)        if v < u_p, else 1
//   a2 = (u_{p+1} - v) / (u_{p+1} - u_1) if v > u_1, else 1
// Children get gamma * a and inherit the coefficient; two B-splines with equal
// knots merge (gamma = ga + gb, c = (ga ca + gb cb) / gamma), so the function
// and the partition of unity are preserved exactly up to rounding.
//
// Elements are boxes [lo, hi); a point lies in the unique element with
// lo <= x < hi per axis, closed at hi = 1.  All knots are dyadic, hence exact
// in FP32 and FP64.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <string>
#include <unordered_map>
#include <vector>

namespace {

constexpr int kMaxP = 4;               // degree bound per axis
constexpr int kMaxK = kMaxP + 2;       // knots per axis per B-spline
constexpr int kMaxComp = 4;

struct Box {
  double lo[3], hi[3];
};

struct BSpl {
  double k[3][kMaxK];
  double gamma;
  double c[kMaxComp];
  bool alive;
  int64_t born;  // refinement number that created it
};

struct Key {
  std::array<double, 3 * kMaxK> v;
  bool operator==(const Key& o) const { return v == o.v; }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = 1469598103934665603ull;
    for (double d : k.v) {
      uint64_t b;
      std::memcpy(&b, &d, 8);
      h ^= b + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    }
    return (size_t)h;
  }
};

struct Gen {
  int p[3];
  int ncomp;
  int G;  // spatial hash: G^3 uniform cells on [0,1]^3
  std::vector<Box> el;
  std::vector<BSpl> bs;
  std::vector<std::vector<int32_t>> ecell, bcell;
  std::unordered_map<Key, int32_t, KeyHash> bmap;
  std::vector<uint32_t> estamp, bstamp;
  uint32_t stamp = 0;
  int64_t n_alive_bs = 0;
  int64_t epoch = 0;
  std::string err;
  std::vector<std::pair<double, double>> iv;
  std::vector<double> cand;

  int cidx(int i, int j, int k) const { return (k * G + j) * G + i; }

  void crange(double lo, double hi, int& a, int& b) const {
    a = (int)std::floor(lo * G);
    b = (int)std::ceil(hi * G) - 1;
    if (a < 0) a = 0;
    if (b > G - 1) b = G - 1;
    if (b < a) b = a;
  }

  Key key_of(const BSpl& s) const {
    Key k;
    k.v.fill(0.0);
    for (int d = 0; d < 3; ++d)
      for (int r = 0; r < p[d] + 2; ++r) k.v[d * kMaxK + r] = s.k[d][r];
    return k;
  }

  void add_elem_cells(int32_t id) {
    const Box& b = el[id];
    int a0, a1, b0, b1, c0, c1;
    crange(b.lo[0], b.hi[0], a0, a1);
    crange(b.lo[1], b.hi[1], b0, b1);
    crange(b.lo[2], b.hi[2], c0, c1);
    for (int k = c0; k <= c1; ++k)
      for (int j = b0; j <= b1; ++j)
        for (int i = a0; i <= a1; ++i) ecell[cidx(i, j, k)].push_back(id);
  }

  // Removes element id from the cells with index c0..c1 on axis ax (within its
  // box on the other axes), after the element shrank on that axis.
  void drop_elem_cells(int32_t id, int ax, int c0, int c1) {
    const Box& b = el[id];
    int r[3][2];
    for (int d = 0; d < 3; ++d) crange(b.lo[d], b.hi[d], r[d][0], r[d][1]);
    r[ax][0] = c0;
    r[ax][1] = c1;
    for (int k = r[2][0]; k <= r[2][1]; ++k)
      for (int j = r[1][0]; j <= r[1][1]; ++j)
        for (int i = r[0][0]; i <= r[0][1]; ++i) {
          auto& v = ecell[cidx(i, j, k)];
          auto it = std::find(v.begin(), v.end(), id);
          if (it != v.end()) {
            *it = v.back();
            v.pop_back();
          }
        }
  }

  void add_bspl_cells(int32_t id) {
    const BSpl& s = bs[id];
    int r[3][2];
    for (int d = 0; d < 3; ++d) crange(s.k[d][0], s.k[d][p[d] + 1], r[d][0], r[d][1]);
    for (int k = r[2][0]; k <= r[2][1]; ++k)
      for (int j = r[1][0]; j <= r[1][1]; ++j)
        for (int i = r[0][0]; i <= r[0][1]; ++i) bcell[cidx(i, j, k)].push_back(id);
  }

  uint32_t next_stamp() {
    if (++stamp == 0) {
      std::fill(estamp.begin(), estamp.end(), 0u);
      std::fill(bstamp.begin(), bstamp.end(), 0u);
      stamp = 1;
    }
    return stamp;
  }

  // Elements overlapping the open box (lo, hi) with positive volume.
  void gather_elems(const double lo[3], const double hi[3], std::vector<int32_t>& out) {
    out.clear();
    uint32_t st = next_stamp();
    if (estamp.size() < el.size()) estamp.resize(el.size() * 2 + 16, 0u);
    int r[3][2];
    for (int d = 0; d < 3; ++d) crange(lo[d], hi[d], r[d][0], r[d][1]);
    for (int k = r[2][0]; k <= r[2][1]; ++k)
      for (int j = r[1][0]; j <= r[1][1]; ++j)
        for (int i = r[0][0]; i <= r[0][1]; ++i)
          for (int32_t id : ecell[cidx(i, j, k)]) {
            if (estamp[id] == st) continue;
            estamp[id] = st;
            const Box& b = el[id];
            bool ov = true;
            for (int d = 0; d < 3; ++d) ov = ov && b.lo[d] < hi[d] && b.hi[d] > lo[d];
            if (ov) out.push_back(id);
          }
  }

  int32_t find_elem(const double q[3]) {
    int c[3];
    for (int d = 0; d < 3; ++d) {
      c[d] = (int)std::floor(q[d] * G);
      if (c[d] > G - 1) c[d] = G - 1;
      if (c[d] < 0) c[d] = 0;
    }
    for (int32_t id : ecell[cidx(c[0], c[1], c[2])]) {
      const Box& b = el[id];
      bool in = true;
      for (int d = 0; d < 3; ++d)
        in = in && b.lo[d] <= q[d] && (q[d] < b.hi[d] || (q[d] == 1.0 && b.hi[d] == 1.0));
      if (in) return id;
    }
    return -1;
  }

  bool supp_contains_box(const BSpl& s, const Box& b) const {
    for (int d = 0; d < 3; ++d)
      if (!(s.k[d][0] <= b.lo[d] && b.hi[d] <= s.k[d][p[d] + 1])) return false;
    return true;
  }

  double supp_volume(const BSpl& s) const {
    double v = 1.0;
    for (int d = 0; d < 3; ++d) v *= s.k[d][p[d] + 1] - s.k[d][0];
    return v;
  }

  bool knots_less(const BSpl& a, const BSpl& b) const {
    for (int d = 0; d < 3; ++d)
      for (int r = 0; r < p[d] + 2; ++r) {
        if (a.k[d][r] < b.k[d][r]) return true;
        if (a.k[d][r] > b.k[d][r]) return false;
      }
    return false;
  }

  int32_t smallest_bspl_over(int32_t eid) {
    const Box& b = el[eid];
    double mid[3];
    for (int d = 0; d < 3; ++d) mid[d] = 0.5 * (b.lo[d] + b.hi[d]);
    int c[3];
    for (int d = 0; d < 3; ++d) {
      c[d] = (int)std::floor(mid[d] * G);
      if (c[d] > G - 1) c[d] = G - 1;
    }
    int32_t best = -1;
    double bestv = 0.0;
    for (int32_t id : bcell[cidx(c[0], c[1], c[2])]) {
      const BSpl& s = bs[id];
      if (!s.alive || !supp_contains_box(s, b)) continue;
      double v = supp_volume(s);
      if (best < 0 || v < bestv || (v == bestv && knots_less(s, bs[best]))) {
        best = id;
        bestv = v;
      }
    }
    return best;
  }

  // Adds a B-spline (or merges into an existing one with the same knots).
  int32_t add_or_merge(const BSpl& s) {
    Key k = key_of(s);
    auto it = bmap.find(k);
    if (it != bmap.end()) {
      BSpl& t = bs[it->second];
      double g = t.gamma + s.gamma;
      for (int q = 0; q < ncomp; ++q) t.c[q] = (t.gamma * t.c[q] + s.gamma * s.c[q]) / g;
      t.gamma = g;
      return it->second;
    }
    int32_t id = (int32_t)bs.size();
    bs.push_back(s);
    bs.back().alive = true;
    bs.back().born = epoch;
    bmap.emplace(k, id);
    if (bstamp.size() < bs.size()) bstamp.resize(bs.size() * 2 + 16, 0u);
    add_bspl_cells(id);
    ++n_alive_bs;
    return id;
  }

  // Finds a mesh plane that traverses the support of s and is not one of its
  // knots: axis ax, value v (smallest axis, then smallest value).  Returns
  // false if s is of minimal support.  A value x strictly inside the support is
  // a traversing plane iff it is an element face and no element inside the
  // support has lo < x < hi on that axis (elements partition the support).
  bool find_traversal(const BSpl& s, std::vector<int32_t>& tmp, int& ax, double& v) {
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = s.k[d][0];
      hi[d] = s.k[d][p[d] + 1];
    }
    gather_elems(lo, hi, tmp);
    for (int d = 0; d < 3; ++d) {
      iv.clear();
      cand.clear();
      for (int32_t id : tmp) {
        const Box& b = el[id];
        iv.emplace_back(b.lo[d], b.hi[d]);
        const double f[2] = {b.lo[d], b.hi[d]};
        for (double x : f) {
          if (!(lo[d] < x && x < hi[d])) continue;
          bool is_knot = false;
          for (int r = 1; r <= p[d]; ++r) is_knot = is_knot || s.k[d][r] == x;
          if (!is_knot) cand.push_back(x);
        }
      }
      if (cand.empty()) continue;
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      std::sort(iv.begin(), iv.end());
      size_t ptr = 0;
      double maxhi = -1.0;
      for (double x : cand) {
        while (ptr < iv.size() && iv[ptr].first < x) maxhi = std::max(maxhi, iv[ptr++].second);
        if (maxhi <= x) {
          ax = d;
          v = x;
          return true;
        }
      }
    }
    return false;
  }

  // True iff the plane x_ax = m traverses the support of s and is not one of
  // its knots: m strictly inside and no element of the support straddles m.
  bool plane_traverses(const BSpl& s, int ax, double m) {
    if (!(s.k[ax][0] < m && m < s.k[ax][p[ax] + 1])) return false;
    for (int r = 1; r <= p[ax]; ++r)
      if (s.k[ax][r] == m) return false;
    uint32_t st = next_stamp();
    int r[3][2];
    for (int d = 0; d < 3; ++d) crange(s.k[d][0], s.k[d][p[d] + 1], r[d][0], r[d][1]);
    r[ax][0] = std::max(0, (int)std::floor(m * G) - 1);
    r[ax][1] = std::min(G - 1, (int)std::floor(m * G));
    for (int k = r[2][0]; k <= r[2][1]; ++k)
      for (int j = r[1][0]; j <= r[1][1]; ++j)
        for (int i = r[0][0]; i <= r[0][1]; ++i)
          for (int32_t id : ecell[cidx(i, j, k)]) {
            if (estamp[id] == st) continue;
            estamp[id] = st;
            const Box& b = el[id];
            if (!(b.lo[ax] < m && m < b.hi[ax])) continue;
            bool inside = true;
            for (int d = 0; d < 3; ++d) inside = inside && b.lo[d] < s.k[d][p[d] + 1] && b.hi[d] > s.k[d][0];
            if (inside) return false;
          }
    return true;
  }

  // Splits queued B-splines until none is traversed by a mesh plane.  B-splines
  // older than the current refinement were of minimal support before the new
  // plane x_ax = m was inserted, so only that plane can traverse them.
  void split_queue(std::deque<int32_t>& q, int new_ax, double new_m) {
    std::vector<int32_t> tmp;
    while (!q.empty()) {
      int32_t id = q.front();
      q.pop_front();
      if (!bs[id].alive) continue;
      int ax;
      double v;
      if (bs[id].born < epoch) {
        if (!plane_traverses(bs[id], new_ax, new_m)) continue;
        ax = new_ax;
        v = new_m;
      } else if (!find_traversal(bs[id], tmp, ax, v)) {
        continue;
      }
      BSpl par = bs[id];
      bs[id].alive = false;
      bmap.erase(key_of(par));
      --n_alive_bs;
      const int pp = p[ax];
      double u[kMaxK], w[kMaxK + 1];
      for (int r = 0; r < pp + 2; ++r) u[r] = par.k[ax][r];
      int n = 0;
      bool ins = false;
      for (int r = 0; r < pp + 2; ++r) {
        if (!ins && v < u[r]) {
          w[n++] = v;
          ins = true;
        }
        w[n++] = u[r];
      }
      if (!ins) w[n++] = v;
      double a1 = (v < u[pp]) ? (v - u[0]) / (u[pp] - u[0]) : 1.0;
      double a2 = (v > u[1]) ? (u[pp + 1] - v) / (u[pp + 1] - u[1]) : 1.0;
      BSpl c1 = par, c2 = par;
      for (int r = 0; r < pp + 2; ++r) {
        c1.k[ax][r] = w[r];
        c2.k[ax][r] = w[r + 1];
      }
      c1.gamma = par.gamma * a1;
      c2.gamma = par.gamma * a2;
      int32_t i1 = add_or_merge(c1);
      int32_t i2 = add_or_merge(c2);
      q.push_back(i1);
      q.push_back(i2);
    }
  }

  // axis < 0: halve the element holding qpt along its longest side (ties
  // x<y<z); otherwise cut it at x_axis = value, which must lie strictly inside.
  bool refine_at(const double qpt[3], int axis = -1, double value = 0.0) {
    ++epoch;
    int32_t e = find_elem(qpt);
    if (e < 0) {
      err = "seed point outside the domain";
      return false;
    }
    Box eb = el[e];
    int ax = 0;
    double m;
    if (axis < 0) {
      double best = eb.hi[0] - eb.lo[0];
      for (int d = 1; d < 3; ++d)
        if (eb.hi[d] - eb.lo[d] > best) {
          best = eb.hi[d] - eb.lo[d];
          ax = d;
        }
      m = 0.5 * (eb.lo[ax] + eb.hi[ax]);
    } else {
      ax = axis;
      m = value;
      if (!(eb.lo[ax] < m && m < eb.hi[ax])) {
        err = "cut value not strictly inside the element";
        return false;
      }
    }
    int32_t ns = smallest_bspl_over(e);
    if (ns < 0) {
      err = "no B-spline covers an element";
      return false;
    }
    const BSpl star = bs[ns];
    double rlo[3], rhi[3];
    for (int d = 0; d < 3; ++d) {
      rlo[d] = star.k[d][0];
      rhi[d] = star.k[d][p[d] + 1];
    }
    // Elements crossed by {x_ax = m} inside the rectangle.
    double glo[3], ghi[3];
    std::memcpy(glo, rlo, sizeof glo);
    std::memcpy(ghi, rhi, sizeof ghi);
    glo[ax] = m;
    ghi[ax] = m;
    std::vector<int32_t> hit;
    {
      // gather_elems needs a positive-width box on ax; widen by one cell and filter.
      double wlo[3], whi[3];
      std::memcpy(wlo, glo, sizeof wlo);
      std::memcpy(whi, ghi, sizeof whi);
      wlo[ax] = std::max(0.0, m - 1.0 / G);
      whi[ax] = std::min(1.0, m + 1.0 / G);
      std::vector<int32_t> cand;
      gather_elems(wlo, whi, cand);
      for (int32_t id : cand) {
        const Box& b = el[id];
        if (!(b.lo[ax] < m && m < b.hi[ax])) continue;
        bool in = true;
        for (int d = 0; d < 3; ++d) {
          if (d == ax) continue;
          if (!(b.lo[d] < rhi[d] && b.hi[d] > rlo[d])) in = false;
        }
        if (!in) continue;
        for (int d = 0; d < 3; ++d) {
          if (d == ax) continue;
          if (b.lo[d] < rlo[d] || b.hi[d] > rhi[d]) {
            err = "mesh rectangle cuts an element partially";
            return false;
          }
        }
        hit.push_back(id);
      }
    }
    for (int32_t id : hit) {
      Box up = el[id];
      up.lo[ax] = m;
      int a0, a1, n0, n1;
      crange(el[id].lo[ax], el[id].hi[ax], a0, a1);
      crange(el[id].lo[ax], m, n0, n1);
      el[id].hi[ax] = m;
      if (n1 < a1) drop_elem_cells(id, ax, n1 + 1, a1);
      int32_t nid = (int32_t)el.size();
      el.push_back(up);
      if (estamp.size() < el.size()) estamp.resize(el.size() * 2 + 16, 0u);
      add_elem_cells(nid);
    }
    // Queue every B-spline whose support the new rectangle meets.
    std::deque<int32_t> q;
    {
      uint32_t st = next_stamp();
      int r[3][2];
      for (int d = 0; d < 3; ++d) {
        if (d == ax) {
          r[d][0] = std::max(0, (int)std::floor(m * G) - 1);
          r[d][1] = std::min(G - 1, (int)std::floor(m * G));
        } else {
          crange(rlo[d], rhi[d], r[d][0], r[d][1]);
        }
      }
      for (int k = r[2][0]; k <= r[2][1]; ++k)
        for (int j = r[1][0]; j <= r[1][1]; ++j)
          for (int i = r[0][0]; i <= r[0][1]; ++i)
            for (int32_t id : bcell[cidx(i, j, k)]) {
              if (bstamp[id] == st) continue;
              bstamp[id] = st;
              const BSpl& s = bs[id];
              if (!s.alive) continue;
              if (!(s.k[ax][0] < m && m < s.k[ax][p[ax] + 1])) continue;
              bool ov = true;
              for (int d = 0; d < 3; ++d) {
                if (d == ax) continue;
                ov = ov && s.k[d][0] < rhi[d] && s.k[d][p[d] + 1] > rlo[d];
              }
              if (ov) q.push_back(id);
            }
      std::sort(q.begin(), q.end());
    }
    split_queue(q, ax, m);
    return true;
  }
};

thread_local std::string g_err;

}  // namespace

extern "C" {

__attribute__((visibility("default"))) const char* lrgen_last_error(void) { return g_err.c_str(); }

// Open tensor mesh n[d] elements per axis, degrees p[d], ncomp coefficient
// components.  Initial B-spline (ix, iy, iz) has id (iz*(ny+py) + iy)*(nx+px) + ix.
__attribute__((visibility("default"))) void* lrgen_create(const int32_t p[3], const int32_t n[3],
                                                          int32_t ncomp, int32_t grid) {
  for (int d = 0; d < 3; ++d)
    if (p[d] < 1 || p[d] > kMaxP || n[d] < 1) {
      g_err = "degree must be in [1,4] and n >= 1";
      return nullptr;
    }
  if (ncomp < 1 || ncomp > kMaxComp || grid < 1) {
    g_err = "ncomp must be in [1,4] and grid >= 1";
    return nullptr;
  }
  Gen* g = new Gen();
  for (int d = 0; d < 3; ++d) g->p[d] = p[d];
  g->ncomp = ncomp;
  g->G = grid;
  g->ecell.resize((size_t)grid * grid * grid);
  g->bcell.resize((size_t)grid * grid * grid);
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i) {
        Box b;
        int ijk[3] = {i, j, k};
        for (int d = 0; d < 3; ++d) {
          b.lo[d] = (double)ijk[d] / n[d];
          b.hi[d] = (double)(ijk[d] + 1) / n[d];
        }
        g->el.push_back(b);
        g->add_elem_cells((int32_t)g->el.size() - 1);
      }
  g->estamp.assign(g->el.size() * 2 + 16, 0u);
  std::vector<double> gk[3];
  for (int d = 0; d < 3; ++d) {
    for (int r = 0; r <= p[d]; ++r) gk[d].push_back(0.0);
    for (int r = 1; r < n[d]; ++r) gk[d].push_back((double)r / n[d]);
    for (int r = 0; r <= p[d]; ++r) gk[d].push_back(1.0);
  }
  const int nb[3] = {n[0] + p[0], n[1] + p[1], n[2] + p[2]};
  for (int k = 0; k < nb[2]; ++k)
    for (int j = 0; j < nb[1]; ++j)
      for (int i = 0; i < nb[0]; ++i) {
        BSpl s;
        std::memset(&s, 0, sizeof s);
        int ijk[3] = {i, j, k};
        for (int d = 0; d < 3; ++d)
          for (int r = 0; r < p[d] + 2; ++r) s.k[d][r] = gk[d][ijk[d] + r];
        s.gamma = 1.0;
        g->add_or_merge(s);
      }
  return g;
}

__attribute__((visibility("default"))) void lrgen_destroy(void* h) { delete (Gen*)h; }

// Sets the coefficients of the initial tensor B-splines ([n_bspl][ncomp]);
// refinement then carries them along so that the function is preserved.
__attribute__((visibility("default"))) int32_t lrgen_set_coef(void* h, const double* c, int64_t n) {
  Gen* g = (Gen*)h;
  if ((int64_t)g->bs.size() != n) {
    g_err = "coefficient count does not match the B-spline count";
    return -1;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int q = 0; q < g->ncomp; ++q) g->bs[i].c[q] = c[i * g->ncomp + q];
  return 0;
}

// Applies one refinement per seed point (points [npts][3], all in [0,1]^3)
// until n_elem >= target_elems or max_ref refinements are done.  Returns the
// number of points consumed, or -1 on error.
__attribute__((visibility("default"))) int64_t lrgen_refine(void* h, const double* pts, int64_t npts,
                                                            int64_t target_elems, int64_t max_ref) {
  Gen* g = (Gen*)h;
  int64_t used = 0;
  while (used < npts && (int64_t)g->el.size() < target_elems && used < max_ref) {
    if (!g->refine_at(pts + 3 * used)) {
      g_err = g->err;
      return -1;
    }
    ++used;
  }
  return used;
}

// One refinement through the element holding q, cut at x_axis = value.
__attribute__((visibility("default"))) int32_t lrgen_refine_plane(void* h, const double q[3], int32_t axis,
                                                                  double value) {
  Gen* g = (Gen*)h;
  if (axis < 0 || axis > 2) {
    g_err = "axis must be 0, 1 or 2";
    return -1;
  }
  if (!g->refine_at(q, axis, value)) {
    g_err = g->err;
    return -1;
  }
  return 0;
}

__attribute__((visibility("default"))) void lrgen_counts(void* h, int64_t* n_elem, int64_t* n_bspl) {
  Gen* g = (Gen*)h;
  *n_elem = (int64_t)g->el.size();
  *n_bspl = g->n_alive_bs;
}

// elem_box [n_elem][6] (lo xyz, hi xyz); knots [n_bspl][3][kstride] with
// kstride = max(p) + 2 (unused tail zero); gamma [n_bspl]; coef [n_bspl][ncomp].
__attribute__((visibility("default"))) void lrgen_export(void* h, double* elem_box, double* knots,
                                                         double* gamma, double* coef) {
  Gen* g = (Gen*)h;
  for (size_t e = 0; e < g->el.size(); ++e)
    for (int d = 0; d < 3; ++d) {
      elem_box[e * 6 + d] = g->el[e].lo[d];
      elem_box[e * 6 + 3 + d] = g->el[e].hi[d];
    }
  const int ks = std::max(g->p[0], std::max(g->p[1], g->p[2])) + 2;
  int64_t o = 0;
  for (const BSpl& s : g->bs) {
    if (!s.alive) continue;
    for (int d = 0; d < 3; ++d)
      for (int r = 0; r < ks; ++r) knots[(o * 3 + d) * ks + r] = r < g->p[d] + 2 ? s.k[d][r] : 0.0;
    gamma[o] = s.gamma;
    for (int q = 0; q < g->ncomp; ++q) coef[o * g->ncomp + q] = s.c[q];
    ++o;
  }
}

}  // extern "C"
