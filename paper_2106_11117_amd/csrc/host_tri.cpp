// Triangle-mesh levels on the host (Sec. 3.1: conforming P1 elements with
// mass lumping on a triangulation; Sec. 3.3: the projector P onto the DOFs of
// the fine elements).  Builds the DOF numbering, the lumped masses, the
// stiffness couplings of every DOF row with the geometric weights of the
// (at most two) triangles that share each edge, the sets P and F+, and the
// fine tiles: a partition of F+ whose regions (the F+ DOFs within graph
// distance p, by increasing distance) run the p substeps of a coarse step in
// one workgroup.
//
// Compiled without floating-point contraction: the areas, masses and weights
// are evaluated with the general P1 formulas in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "host.h"

namespace lts {

namespace {

// Interleaved bits of two 16-bit coordinates (Morton order).
uint32_t morton16(uint32_t x, uint32_t y) {
  auto spread = [](uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
  };
  return spread(x) | (spread(y) << 1);
}

}  // namespace

std::string build_tri(const lts_mesh_desc& d, TriHost& T) {
  T = TriHost();
  const int nn = d.n_nodes, nt = d.n_tris;
  if (nn < 3 || nt < 1) return "need n_nodes >= 3 and n_tris >= 1";
  if (!d.xy || !d.tri || !d.tri_block) return "xy, tri and tri_block are required";
  if (d.n_blocks < 1 || d.n_blocks > 255) return "n_blocks must be in 1..255";
  if (d.p < 1 || d.p > 64) return "p must be in 1..64";
  if (!(d.nu >= 0.0 && d.nu <= 1.0)) return "nu must be in [0, 1]";
  if (!(d.h > 0.0) || !std::isfinite(d.h)) return "h must be finite and > 0";
  for (int i = 0; i < 2 * nn; ++i)
    if (!std::isfinite(d.xy[i])) return "xy must be finite";
  if (d.qoi_w)
    for (int i = 0; i < nn; ++i)
      if (!std::isfinite(d.qoi_w[i])) return "qoi_w must be finite";
  T.n_nodes = nn;
  T.n_tris = nt;
  // ---- triangles: indices, orientation, blocks; twice the area
  std::vector<double> twoA(nt);
  for (int t = 0; t < nt; ++t) {
    const int* v = d.tri + 3 * (size_t)t;
    for (int k = 0; k < 3; ++k)
      if (v[k] < 0 || v[k] >= nn) return "triangle node index out of range";
    if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2]) return "triangle with a repeated node";
    if (d.tri_block[t] < 0 || d.tri_block[t] >= d.n_blocks) return "tri_block out of range";
    const double x0 = d.xy[2 * v[0]], y0 = d.xy[2 * v[0] + 1];
    const double x1 = d.xy[2 * v[1]], y1 = d.xy[2 * v[1] + 1];
    const double x2 = d.xy[2 * v[2]], y2 = d.xy[2 * v[2] + 1];
    twoA[t] = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
    if (!(twoA[t] > 0.0)) return "triangle not counter-clockwise (area <= 0)";
  }
  // ---- DOFs: not Dirichlet; each must be a vertex of a triangle
  std::vector<uint8_t> in_tri(nn, 0);
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) in_tri[d.tri[3 * (size_t)t + k]] = 1;
  std::vector<int> dofs;
  for (int i = 0; i < nn; ++i) {
    const bool dir = d.dirichlet && d.dirichlet[i];
    if (dir) continue;
    if (!in_tri[i]) return "a node that is not Dirichlet belongs to no triangle";
    dofs.push_back(i);
  }
  if (dofs.empty()) return "the mesh has no DOF";
  // Morton order of the DOF coordinates (ties: node id)
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  for (int i : dofs) {
    xmin = std::min(xmin, d.xy[2 * i]);
    xmax = std::max(xmax, d.xy[2 * i]);
    ymin = std::min(ymin, d.xy[2 * i + 1]);
    ymax = std::max(ymax, d.xy[2 * i + 1]);
  }
  const double sx = xmax > xmin ? 65535.0 / (xmax - xmin) : 0.0, sy = ymax > ymin ? 65535.0 / (ymax - ymin) : 0.0;
  std::vector<std::pair<uint32_t, int>> key;
  key.reserve(dofs.size());
  for (int i : dofs)
    key.push_back({morton16((uint32_t)((d.xy[2 * i] - xmin) * sx), (uint32_t)((d.xy[2 * i + 1] - ymin) * sy)), i});
  std::sort(key.begin(), key.end());
  const int n = (int)key.size();
  T.n_dof = n;
  T.node_dof.assign(nn, -1);
  T.dof_node.resize(n);
  for (int k = 0; k < n; ++k) {
    T.dof_node[k] = key[k].second;
    T.node_dof[key[k].second] = k;
  }
  // ---- lumped mass: m_i = (sum over triangles T containing i of 2|T|) / 6
  std::vector<double> twoAsum(nn, 0.0);
  for (int k = 0; k < 3; ++k)                 // vertex slot by slot, triangles in order
    for (int t = 0; t < nt; ++t) twoAsum[d.tri[3 * (size_t)t + k]] += twoA[t];
  T.mass_node.resize(nn);
  for (int i = 0; i < nn; ++i) T.mass_node[i] = twoAsum[i] / 6.0;
  // ---- couplings: per undirected edge the (block, -|T| grad l_a . grad l_b)
  //      of each triangle that has it
  struct EdgeTris {
    int blk[2] = {255, 255};
    double w[2] = {0.0, 0.0};
    int n = 0;
  };
  std::map<std::pair<int, int>, EdgeTris> edges;
  for (int t = 0; t < nt; ++t) {
    const int* v = d.tri + 3 * (size_t)t;
    double x[3], y[3];
    for (int k = 0; k < 3; ++k) {
      x[k] = d.xy[2 * v[k]];
      y[k] = d.xy[2 * v[k] + 1];
    }
    const double area = 0.5 * std::fabs(twoA[t]);
    const double gx[3] = {(y[1] - y[2]) / twoA[t], (y[2] - y[0]) / twoA[t], (y[0] - y[1]) / twoA[t]};
    const double gy[3] = {(x[2] - x[1]) / twoA[t], (x[0] - x[2]) / twoA[t], (x[1] - x[0]) / twoA[t]};
    for (int a = 0; a < 3; ++a)
      for (int b = a + 1; b < 3; ++b) {
        const double geo = area * (gx[a] * gx[b] + gy[a] * gy[b]);
        const std::pair<int, int> e{std::min(v[a], v[b]), std::max(v[a], v[b])};
        EdgeTris& E = edges[e];
        if (E.n == 2) return "an edge belongs to more than two triangles";
        E.blk[E.n] = d.tri_block[t];
        E.w[E.n] = -geo;
        ++E.n;
      }
  }
  // rows of the DOFs: neighbours in increasing DOF index, Dirichlet ones last
  std::vector<std::vector<std::pair<int, const EdgeTris*>>> nb(n);
  for (const auto& kv : edges) {
    const int a = kv.first.first, b = kv.first.second;
    const int da = T.node_dof[a], db = T.node_dof[b];
    if (da >= 0) nb[da].push_back({db >= 0 ? db : n, &kv.second});
    if (db >= 0) nb[db].push_back({da >= 0 ? da : n, &kv.second});
  }
  T.rp.assign(n + 1, 0);
  for (int k = 0; k < n; ++k) {
    std::stable_sort(nb[k].begin(), nb[k].end(),
                     [](const std::pair<int, const EdgeTris*>& x, const std::pair<int, const EdgeTris*>& y) {
                       return x.first < y.first;
                     });
    T.rp[k + 1] = T.rp[k] + (int)nb[k].size();
  }
  const int nnz = T.rp[n];
  T.col.resize(nnz);
  T.eblk.resize(nnz);
  T.ewa.resize(nnz);
  T.ewb.resize(nnz);
  for (int k = 0; k < n; ++k)
    for (size_t e = 0; e < nb[k].size(); ++e) {
      const int o = T.rp[k] + (int)e;
      const EdgeTris& E = *nb[k][e].second;
      T.col[o] = nb[k][e].first;
      T.eblk[o] = E.blk[0] | (E.blk[1] << 8);
      T.ewa[o] = E.w[0];
      T.ewb[o] = E.w[1];
    }
  // ---- P: DOFs that are vertices of a fine element; F+: P and the DOFs
  //      coupled to P by a nonzero entry of K (unit coefficient)
  T.dflag.assign(n + 1, 0);
  if (d.tri_fine)
    for (int t = 0; t < nt; ++t)
      if (d.tri_fine[t])
        for (int k = 0; k < 3; ++k) {
          const int q = T.node_dof[d.tri[3 * (size_t)t + k]];
          if (q >= 0) T.dflag[q] |= 1;
        }
  for (int k = 0; k < n; ++k) {
    if (T.dflag[k] & 1) {
      T.dflag[k] |= 2;
      continue;
    }
    for (int o = T.rp[k]; o < T.rp[k + 1]; ++o) {
      const int j = T.col[o];
      // K_kj with kappa = 1: the summed element entries of the edge (minus the weights)
      if (j < n && (T.dflag[j] & 1) && (T.ewa[o] + T.ewb[o]) != 0.0) {
        T.dflag[k] |= 2;
        break;
      }
    }
  }
  T.node_flags.assign(nn, 0);
  T.dx.resize(n);
  T.dy.resize(n);
  T.invm.resize(n);
  T.qoiw.resize(n);
  for (int k = 0; k < n; ++k) {
    const int i = T.dof_node[k];
    T.dx[k] = d.xy[2 * i];
    T.dy[k] = d.xy[2 * i + 1];
    T.invm[k] = 1.0 / T.mass_node[i];
    T.qoiw[k] = d.qoi_w ? d.qoi_w[i] : 0.0;
    T.node_flags[i] = LTS_NODE_DOF | ((T.dflag[k] & 1) ? LTS_NODE_P : 0) | ((T.dflag[k] & 2) ? LTS_NODE_FPLUS : 0);
    if (T.dflag[k] & 1) ++T.n_P;
    if (T.dflag[k] & 2) {
      ++T.n_F;
      T.max_deg = std::max(T.max_deg, T.rp[k + 1] - T.rp[k]);
    } else {
      T.coarse.push_back(k);
    }
  }
  if (T.max_deg > kTriMaxDeg) return "an F+ DOF has more than LTS_MESH_MAX_DEGREE stiffness neighbours";
  // ---- fine tiles: recursive bisection of F+ (median of the longer
  //      coordinate extent) until the region of every part fits
  const int p = d.p;
  std::vector<int> F;
  for (int k = 0; k < n; ++k)
    if (T.dflag[k] & 2) F.push_back(k);
  std::vector<int> dist(n + 1, -1), touched;
  // region of a part: F+ DOFs within graph distance p (BFS inside F+),
  // ordered by distance; returns false once it exceeds the cap
  auto region = [&](const std::vector<int>& part, std::vector<int>& out) {
    out.clear();
    for (int k : touched) dist[k] = -1;
    touched.clear();
    for (int k : part) {
      dist[k] = 0;
      touched.push_back(k);
      out.push_back(k);
    }
    if ((int)out.size() > kTriRegionCap) return false;
    for (size_t h = 0; h < out.size(); ++h) {
      const int k = out[h];
      if (dist[k] == p) continue;
      for (int o = T.rp[k]; o < T.rp[k + 1]; ++o) {
        const int j = T.col[o];
        if (j >= n || !(T.dflag[j] & 2) || dist[j] >= 0) continue;
        dist[j] = dist[k] + 1;
        touched.push_back(j);
        out.push_back(j);
        if ((int)out.size() > kTriRegionCap) return false;
      }
    }
    return true;
  };
  T.tiles.push_back(0);
  size_t n_region = 0;
  std::vector<int> reg;
  // the tile of a part whose region is in reg: entries and coupling slots
  auto emit = [&](const std::vector<int>& reg) {
    const int len = (int)reg.size();
    std::map<int, int> loc;
    for (int l = 0; l < len; ++l) loc[reg[l]] = l;
    for (int l = 0; l < len; ++l) {
      const int k = reg[l];
      const int deg = T.rp[k + 1] - T.rp[k];
      TriEnt e;
      e.dof = k | ((T.dflag[k] & 1) ? (int32_t)0x80000000u : 0);
      e.row = T.rp[k];
      e.deg_dist = deg | (dist[k] << 16);
      e.slot0 = (int)T.tslot.size();
      for (int o = T.rp[k]; o < T.rp[k + 1]; ++o) {
        const int j = T.col[o];
        int s = len;
        if (j < n && (T.dflag[j] & 1)) {
          auto it = loc.find(j);
          if (it != loc.end()) s = it->second;
        }
        T.tslot.push_back((uint16_t)s);
      }
      T.ent.push_back(e);
    }
    T.tiles.push_back((int)T.ent.size());
    T.max_region = std::max(T.max_region, len);
    n_region += (size_t)len;
  };
  // Square bins of side b (F+ coordinates binned from the F+ bounding box):
  // the total region size if every bin's region fits, else 0.  The best of a
  // few sides is kept; recursive bisection is the fallback.
  double fx0 = 1e300, fx1 = -1e300, fy0 = 1e300, fy1 = -1e300;
  for (int k : F) {
    fx0 = std::min(fx0, T.dx[k]);
    fx1 = std::max(fx1, T.dx[k]);
    fy0 = std::min(fy0, T.dy[k]);
    fy1 = std::max(fy1, T.dy[k]);
  }
  auto bins = [&](double b, double shift, std::vector<std::vector<int>>& parts) {
    parts.clear();
    const double ox = fx0 - shift * b, oy = fy0 - shift * b;
    const long long nbx = (long long)std::floor((fx1 - ox) / b) + 1, nby = (long long)std::floor((fy1 - oy) / b) + 1;
    if (nbx * nby > (long long)8 * F.size() + 64) return false;   // bins far sparser than F+: not a candidate
    std::map<long long, int> idx;
    for (int k : F) {
      const long long bx = (long long)std::floor((T.dx[k] - ox) / b), by = (long long)std::floor((T.dy[k] - oy) / b);
      auto it = idx.emplace(by * nbx + bx, (int)parts.size());
      if (it.second) parts.emplace_back();
      parts[it.first->second].push_back(k);
    }
    return true;
  };
  double best_b = 0.0, best_shift = 0.0;
  size_t best_total = 0;
  if (!F.empty()) {
    // sides in units of the typical F+ spacing: the median length of the
    // couplings between F+ DOFs
    std::vector<double> len;
    for (int k : F)
      for (int o = T.rp[k]; o < T.rp[k + 1]; ++o) {
        const int j = T.col[o];
        if (j < n && (T.dflag[j] & 2) && j > k) len.push_back(std::hypot(T.dx[j] - T.dx[k], T.dy[j] - T.dy[k]));
      }
    double sp = std::sqrt(std::max((fx1 - fx0) * (fy1 - fy0), 1e-300) / (double)F.size());
    if (!len.empty()) {
      std::nth_element(len.begin(), len.begin() + len.size() / 2, len.end());
      sp = len[len.size() / 2];
    }
    std::vector<std::vector<int>> parts;
    for (double f = std::max(2.0, 0.5 * p); f <= std::sqrt((double)kTriRegionCap); f *= 1.15)
      for (double shift : {0.0, 0.5}) {
        const double b = f * sp;
        if (!bins(b, shift, parts)) continue;
        size_t tot = 0;
        bool ok = true;
        for (auto& pt : parts) {
          if (!region(pt, reg)) {
            ok = false;
            break;
          }
          tot += reg.size();
        }
        if (ok && (best_b == 0.0 || tot < best_total)) {
          best_b = b;
          best_shift = shift;
          best_total = tot;
        }
      }
  }
  std::function<std::string(std::vector<int>&)> bisect = [&](std::vector<int>& part) -> std::string {
    if (part.empty()) return "";
    if (region(part, reg)) {
      emit(reg);
      return "";
    }
    if (part.size() == 1) return "an F+ region exceeds LTS_MESH_REGION_CAP even for a one-DOF tile (p too large)";
    double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
    for (int k : part) {
      x0 = std::min(x0, T.dx[k]);
      x1 = std::max(x1, T.dx[k]);
      y0 = std::min(y0, T.dy[k]);
      y1 = std::max(y1, T.dy[k]);
    }
    const bool by_x = (x1 - x0) >= (y1 - y0);
    std::vector<int> s = part;
    const size_t mid = s.size() / 2;
    std::nth_element(s.begin(), s.begin() + mid, s.end(), [&](int a, int b) {
      const double va = by_x ? T.dx[a] : T.dy[a], vb = by_x ? T.dx[b] : T.dy[b];
      return va < vb || (va == vb && a < b);
    });
    std::vector<int> A(s.begin(), s.begin() + mid), B(s.begin() + mid, s.end());
    std::string e = bisect(A);
    if (!e.empty()) return e;
    return bisect(B);
  };
  // recursive bisection, kept unless the best bins need fewer region nodes
  std::vector<int> all = F;
  const std::string e = bisect(all);
  if (!e.empty() && best_b == 0.0) return e;
  if (best_b > 0.0 && (!e.empty() || best_total < n_region)) {
    T.tiles.assign(1, 0);
    T.ent.clear();
    T.tslot.clear();
    T.max_region = 0;
    n_region = 0;
    std::vector<std::vector<int>> parts;
    bins(best_b, best_shift, parts);
    for (auto& pt : parts) {
      region(pt, reg);
      emit(reg);
    }
  }
  T.halo_ratio = T.n_F ? (double)n_region / T.n_F : 1.0;
  // ---- the header the sample staging needs
  HostLevel& S = T.shell;
  S.n_blocks = d.n_blocks;
  S.h = d.h;
  S.p = p;
  S.nu = d.nu;
  S.n_dof = n;
  S.n_P = T.n_P;
  S.n_F = T.n_F;
  cheb_constants(p, d.nu, S.delta, S.omega, S.beta, S.beta_half);
  return "";
}

}  // namespace lts
