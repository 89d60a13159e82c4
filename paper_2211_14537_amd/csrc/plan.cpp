// Host side of a plan: the box hierarchy over the caller's leaves, the VFMM
// interaction lists, the extension lists and the per-cut-leaf operators.
//
// Section 4 (data structures): a level-restricted quad-tree; colleagues,
// coarse and fine neighbours; the lists of the adaptive VFMM shown in the
// tree-levels figure: n/n+/n- (list 1, near field by tables), i (list 2,
// M2L), i- (list 3: children of colleagues that do not touch a leaf,
// multipole evaluated at its targets) and i+ (list 4: a coarse leaf that is a
// colleague of the parent but does not touch the box, turned into a local
// expansion).  Extension lists: for a cut square S, the exterior leaves that
// Sbar overlaps and whose closest cut-square centre is that of S, the later
// cut square taking precedence on ties; the extension restriction forbids a
// coarser leaf in such a list.
#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cstring>
#include <unordered_map>

#include "vfx_internal.h"

namespace vfx {

namespace {

inline uint64_t key(int l, int x, int y) {
  return ((uint64_t)l << 58) | ((uint64_t)(uint32_t)x << 29) | (uint64_t)(uint32_t)y;
}

inline uint64_t morton(uint32_t x, uint32_t y) {
  uint64_t r = 0;
  for (int b = 0; b < 30; ++b) {
    r |= (uint64_t)((x >> b) & 1u) << (2 * b);
    r |= (uint64_t)((y >> b) & 1u) << (2 * b + 1);
  }
  return r;
}

struct Node {
  int l, x, y, leaf;
};

// closed boxes (la,ax,ay) and (lb,bx,by) touch or overlap
inline bool touch(int la, int ax, int ay, int lb, int bx, int by) {
  const int L = std::max(la, lb);
  const int64_t sa = 1LL << (L - la), sb = 1LL << (L - lb);
  const int64_t ax0 = ax * sa, ax1 = ax0 + sa, ay0 = ay * sa, ay1 = ay0 + sa;
  const int64_t bx0 = bx * sb, bx1 = bx0 + sb, by0 = by * sb, by1 = by0 + sb;
  return ax0 <= bx1 && bx0 <= ax1 && ay0 <= by1 && by0 <= ay1;
}

}  // namespace

// List-1 pairs grouped for the near-field kernels: configuration-major, and
// inside a configuration by precision class (modes 1, 2: sources at level >=
// min_level are applied in mixed precision: the self operator densely, the
// other configurations in their low-rank form, so a configuration without
// one stays in FP64), then by target.  Tiles of <= 64
// pairs go to the low-rank or the dense kernel of their class.  l1_slot maps
// every per-target list-1 entry to its pair.
int build_near_tiles(const Tables& T, HostPlan& H, int mode, int min_level, std::string& err) {
  const int L = H.L;
  const int N1 = H.l1_ptr[L];
  const bool k16 = T.n == 256 && !T.lr_R.empty();
  if (mode >= 1 && !k16) {
    err = "mixed precision is available for K = 16 only";
    return VFX_EINVAL;
  }
  auto mixed = [&](int e) {
    const int c = H.l1_cfg[e];
    return mode >= 1 && H.box_level[H.leaf_box[H.l1_src[e]]] >= min_level && (c == kNearSelf || T.lr_R[c] > 0);
  };
  // counting sort on (configuration, class)
  std::vector<int> cnt(2 * kNearConfigs + 1, 0);
  for (int e = 0; e < N1; ++e) cnt[2 * H.l1_cfg[e] + (mixed(e) ? 1 : 0) + 1]++;
  for (int g = 0; g < 2 * kNearConfigs; ++g) cnt[g + 1] += cnt[g];
  H.np_src.assign(N1, 0);
  H.np_tgt.assign(N1, 0);
  H.l1_slot.assign(N1, 0);
  std::vector<int> pos(cnt.begin(), cnt.end() - 1);
  for (int leaf = 0; leaf < L; ++leaf)  // targets ascending inside each group
    for (int e = H.l1_ptr[leaf]; e < H.l1_ptr[leaf + 1]; ++e) {
      const int s = pos[2 * H.l1_cfg[e] + (mixed(e) ? 1 : 0)]++;
      H.np_src[s] = H.l1_src[e];
      H.np_tgt[s] = leaf;
      H.l1_slot[e] = s;
    }
  for (auto* v : {&H.nt_cfg, &H.nt_first, &H.nt_count, &H.nl_cfg, &H.nl_first, &H.nl_count, &H.mt_cfg,
                  &H.mt_first, &H.mt_count, &H.ml_cfg, &H.ml_first, &H.ml_count})
    v->clear();
  // With the target-stationary near field selected (near_mode 1), FP64 at
  // K = 16 (also precision modes 1, 2 when no pair is mixed) takes that path: every non-self pair's factor product by the
  // table GEMM (configuration-major tiles of 64), then the per-target-group
  // kernel; the self pairs only there
  bool any_mixed = false;
  for (int e = 0; e < N1 && !any_mixed; ++e) any_mixed = mixed(e);
  const bool ts = H.near_mode == 1 && !any_mixed && k16 && T.ts_ok;
  constexpr int kTile = 64;
  for (int c = 0; c < kNearConfigs; ++c) {
    const bool lr = ts ? c != kNearSelf : (k16 && T.lr_R[c] > 0);
    if (ts && !lr) continue;
    for (int cls = 0; cls < 2; ++cls) {
      const int g = 2 * c + cls;
      std::vector<int>*cf, *fi, *co;
      if (cls == 0) {
        cf = lr ? &H.nl_cfg : &H.nt_cfg;
        fi = lr ? &H.nl_first : &H.nt_first;
        co = lr ? &H.nl_count : &H.nt_count;
      } else {
        cf = lr ? &H.ml_cfg : &H.mt_cfg;
        fi = lr ? &H.ml_first : &H.mt_first;
        co = lr ? &H.ml_count : &H.mt_count;
      }
      // FP64 low-rank tiles of the fused kernel hold 32 pairs (it splits a
      // tile's work over its four waves), the others 64
      const int tile = (cls == 0 && lr && !ts) ? kTile / 2 : kTile;
      for (int f = cnt[g]; f < cnt[g + 1]; f += tile) {
        cf->push_back(c);
        fi->push_back(f);
        co->push_back(std::min(tile, cnt[g + 1] - f));
      }
    }
  }
  for (auto* v : {&H.ts_grp, &H.ts_tcls, &H.ts_row, &H.ts_code}) v->clear();
  H.ts = ts;
  if (ts) {
    // per group of kTsGroup targets: the self tile (if any target is a
    // source of its own), then per class as many tiles as the largest
    // number of that class's pairs of one target; tile j of a class holds
    // the j-th such pair of every target (list order), in its target's slot
    std::vector<int> per[kNearClasses];
    for (int t0 = 0; t0 < L; t0 += kTsGroup) {
      const int t1 = std::min(L, t0 + kTsGroup);
      H.ts_grp.push_back((int)H.ts_tcls.size());
      for (int k = 0; k < kNearClasses; ++k) per[k].assign((size_t)kTsGroup * 64, -1);
      int cnt[kNearClasses][kTsGroup] = {};
      for (int t = t0; t < t1; ++t)
        for (int e = H.l1_ptr[t]; e < H.l1_ptr[t + 1]; ++e) {
          const int c = H.l1_cfg[e];
          const int k = T.near_cls[c];
          int& m = cnt[k][t - t0];
          if (m >= 64) {
            err = "near field: more than 64 pairs of one class for a target";
            return VFX_ETREE;
          }
          per[k][(size_t)m * kTsGroup + (t - t0)] = e;
          m++;
        }
      for (int k = 0; k < kNearClasses; ++k) {
        int rounds = 0;
        for (int s = 0; s < kTsGroup; ++s) rounds = std::max(rounds, cnt[k][s]);
        for (int j = 0; j < rounds; ++j) {
          H.ts_tcls.push_back(k);
          for (int s = 0; s < kTsGroup; ++s) {
            const int e = per[k][(size_t)j * kTsGroup + s];
            if (e < 0) {
              H.ts_row.push_back(-1);
              H.ts_code.push_back(0);
            } else if (k == 0) {
              H.ts_row.push_back(H.l1_src[e]);
              H.ts_code.push_back(0);
            } else {
              H.ts_row.push_back(H.l1_slot[e]);
              H.ts_code.push_back(d4_inverse(T.near_g[H.l1_cfg[e]]));
            }
          }
        }
      }
    }
    H.ts_grp.push_back((int)H.ts_tcls.size());
  }
  H.precision = mode;
  H.mixed_min_level = min_level;
  return VFX_OK;
}

int build_host_plan(const Tables& T, const vfx_tree* tree, HostPlan& H, std::string& err, bool defer_factor) {
  auto t0 = std::chrono::steady_clock::now();
  const int L = tree->n_leaves;
  if (L <= 0 || !tree->level || !tree->ix || !tree->iy || !tree->kind) {
    err = "tree: empty or null arrays";
    return VFX_EINVAL;
  }
  H = HostPlan();
  H.L = L;
  std::unordered_map<uint64_t, int> idx;  // key -> node id (before sorting)
  std::vector<Node> nodes;
  nodes.reserve(2 * L);
  int lmax = 0;
  for (int i = 0; i < L; ++i) {
    const int l = tree->level[i], x = tree->ix[i], y = tree->iy[i];
    if (l < 0 || l > 28 || x < 0 || y < 0 || x >= (1 << l) || y >= (1 << l)) {
      err = "tree: leaf " + std::to_string(i) + " has level/position out of range";
      return VFX_EINVAL;
    }
    const int k = tree->kind[i];
    if (k < 0 || k > 2) {
      err = "tree: leaf " + std::to_string(i) + " has an invalid kind";
      return VFX_EINVAL;
    }
    if (!idx.emplace(key(l, x, y), (int)nodes.size()).second) {
      err = "tree: duplicate leaf " + std::to_string(i);
      return VFX_ETREE;
    }
    nodes.push_back({l, x, y, i});
    lmax = std::max(lmax, l);
  }
  // ancestors
  for (int i = 0; i < L; ++i) {
    int l = tree->level[i], x = tree->ix[i], y = tree->iy[i];
    while (l > 0) {
      --l;
      x >>= 1;
      y >>= 1;
      auto it = idx.find(key(l, x, y));
      if (it != idx.end()) {
        if (nodes[it->second].leaf >= 0) {
          err = "tree: leaf " + std::to_string(nodes[it->second].leaf) + " contains another leaf";
          return VFX_ETREE;
        }
        break;  // this ancestor and all above already present
      }
      idx.emplace(key(l, x, y), (int)nodes.size());
      nodes.push_back({l, x, y, -1});
    }
  }
  // every internal node has its four children
  for (const Node& nd : nodes) {
    if (nd.leaf >= 0) continue;
    for (int c = 0; c < 4; ++c)
      if (!idx.count(key(nd.l + 1, 2 * nd.x + c / 2, 2 * nd.y + c % 2))) {
        err = "tree: leaves do not tile the root box (box at level " + std::to_string(nd.l) +
              " misses a child)";
        return VFX_ETREE;
      }
  }
  if (!idx.count(key(0, 0, 0))) {
    err = "tree: no root";
    return VFX_ETREE;
  }
  // order: level-major, Morton within a level
  std::vector<int> order(nodes.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    if (nodes[a].l != nodes[b].l) return nodes[a].l < nodes[b].l;
    return morton(nodes[a].x, nodes[a].y) < morton(nodes[b].x, nodes[b].y);
  });
  const int B = (int)nodes.size();
  H.B = B;
  H.nlev = lmax + 1;
  std::vector<int> newid(B);
  for (int i = 0; i < B; ++i) newid[order[i]] = i;
  for (auto& kv : idx) kv.second = newid[kv.second];
  H.box_level.resize(B);
  H.box_ix.resize(B);
  H.box_iy.resize(B);
  H.box_leaf.resize(B);
  H.box_parent.assign(B, -1);
  H.box_child0.assign(B, -1);
  H.box_cx.resize(B);
  H.box_cy.resize(B);
  H.level_start.assign(H.nlev + 1, 0);
  H.leaf_box.assign(L, -1);
  for (int i = 0; i < B; ++i) {
    const Node& nd = nodes[order[i]];
    H.box_level[i] = nd.l;
    H.box_ix[i] = nd.x;
    H.box_iy[i] = nd.y;
    H.box_leaf[i] = nd.leaf;
    const double h = std::ldexp(T.root_size, -nd.l);
    H.box_cx[i] = T.root_cx - 0.5 * T.root_size + (nd.x + 0.5) * h;
    H.box_cy[i] = T.root_cy - 0.5 * T.root_size + (nd.y + 0.5) * h;
    H.level_start[nd.l + 1]++;
    if (nd.leaf >= 0) H.leaf_box[nd.leaf] = i;
  }
  for (int l = 0; l < H.nlev; ++l) H.level_start[l + 1] += H.level_start[l];
  auto find = [&](int l, int x, int y) -> int {
    if (l < 0 || x < 0 || y < 0 || x >= (1 << l) || y >= (1 << l)) return -1;
    auto it = idx.find(key(l, x, y));
    return it == idx.end() ? -1 : it->second;
  };
  for (int i = 0; i < B; ++i) {
    const int l = H.box_level[i];
    if (l > 0) H.box_parent[i] = find(l - 1, H.box_ix[i] >> 1, H.box_iy[i] >> 1);
    if (H.box_leaf[i] < 0) H.box_child0[i] = find(l + 1, 2 * H.box_ix[i], 2 * H.box_iy[i]);
  }
  // children of a box are contiguous in the Morton order of the next level
  for (int i = 0; i < B; ++i)
    if (H.box_child0[i] >= 0)
      for (int c = 0; c < 4; ++c) {
        const int ch = H.box_child0[i] + c;
        if (ch >= B || H.box_parent[ch] != i) {
          err = "internal: children not contiguous";
          return VFX_EINVAL;
        }
      }
  H.kind.assign(tree->kind, tree->kind + L);

  // ---- extension lists ---------------------------------------------------
  H.owner.assign(L, -1);
  std::vector<int64_t> best(L, -1);
  const int sh = lmax;  // centres in units of root/2^(lmax+1): (2x+1) << (lmax-l)
  auto cen = [&](int b, int64_t* cx, int64_t* cy) {
    *cx = (int64_t)(2 * H.box_ix[b] + 1) << (sh - H.box_level[b]);
    *cy = (int64_t)(2 * H.box_iy[b] + 1) << (sh - H.box_level[b]);
  };
  std::vector<int> stack, cand;
  for (int leaf = 0; leaf < L; ++leaf) {
    if (H.kind[leaf] != 2) continue;
    H.cut_leaf.push_back(leaf);
    H.owner[leaf] = leaf;
    const int b = H.leaf_box[leaf];
    const int l = H.box_level[b], x = H.box_ix[b], y = H.box_iy[b];
    int64_t scx, scy;
    cen(b, &scx, &scy);
    cand.clear();
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        if (dx == 0 && dy == 0) continue;
        const int cx = x + dx, cy = y + dy;
        if (cx < 0 || cy < 0 || cx >= (1 << l) || cy >= (1 << l)) continue;
        const int c = find(l, cx, cy);
        if (c >= 0) {
          stack.assign(1, c);
          while (!stack.empty()) {
            const int u = stack.back();
            stack.pop_back();
            if (H.box_leaf[u] >= 0)
              cand.push_back(H.box_leaf[u]);
            else
              for (int q = 0; q < 4; ++q) stack.push_back(H.box_child0[u] + q);
          }
        } else {
          const int p = find(l - 1, cx >> 1, cy >> 1);
          if (p >= 0 && H.box_leaf[p] >= 0) cand.push_back(H.box_leaf[p]);
        }
      }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    for (int j : cand) {
      if (H.kind[j] != 0) continue;
      int64_t jx, jy;
      cen(H.leaf_box[j], &jx, &jy);
      const int64_t d2 = (jx - scx) * (jx - scx) + (jy - scy) * (jy - scy);
      if (best[j] < 0 || d2 <= best[j]) {
        best[j] = d2;
        H.owner[j] = leaf;
      }
    }
  }
  H.ncut = (int)H.cut_leaf.size();
  std::vector<int> cutpos(L, -1);
  for (int c = 0; c < H.ncut; ++c) cutpos[H.cut_leaf[c]] = c;
  std::vector<std::vector<int>> tg(H.ncut);
  for (int c = 0; c < H.ncut; ++c) tg[c].push_back(H.cut_leaf[c]);
  for (int j = 0; j < L; ++j) {
    if (H.kind[j] != 0 || H.owner[j] < 0) continue;
    const int s = H.owner[j];
    if (H.box_level[H.leaf_box[s]] > H.box_level[H.leaf_box[j]]) {
      err = "tree: extension restriction violated (cut leaf " + std::to_string(s) +
            " would extend onto the coarser leaf " + std::to_string(j) + ")";
      return VFX_ETREE;
    }
    tg[cutpos[s]].push_back(j);
  }
  H.ext_ptr.assign(H.ncut + 1, 0);
  for (int c = 0; c < H.ncut; ++c) {
    H.ext_ptr[c + 1] = H.ext_ptr[c] + (int)tg[c].size();
    H.ext_tgt.insert(H.ext_tgt.end(), tg[c].begin(), tg[c].end());
    // target grid in the cut leaf's Sbar frame (Sbar = 3x the cut leaf,
    // same centre): node a of target j sits at o + s t_a per axis
    const int bS = H.leaf_box[H.cut_leaf[c]];
    const double hS = std::ldexp(T.root_size, -H.box_level[bS]);
    for (int j : tg[c]) {
      const int bj = H.leaf_box[j];
      const double hj = std::ldexp(T.root_size, -H.box_level[bj]);
      H.ext_geo.push_back((H.box_cx[bj] - H.box_cx[bS]) / (1.5 * hS));
      H.ext_geo.push_back((H.box_cy[bj] - H.box_cy[bS]) / (1.5 * hS));
      H.ext_geo.push_back(hj / (3.0 * hS));
    }
  }

  // ---- sources whose data are identically zero ------------------------------
  // f^e vanishes on an exterior leaf outside every extension list, whatever
  // f is, so such a leaf (and a box all of whose leaves are such) adds
  // exactly zero to every potential: it is left out as a source of lists 1-4
  // (it stays a target).
  std::vector<uint8_t> zero_leaf(L, 0), zero_box(B, 1);
  for (int j = 0; j < L; ++j) zero_leaf[j] = (H.kind[j] == 0 && H.owner[j] < 0) ? 1 : 0;
  for (int l = H.nlev - 1; l >= 0; --l)
    for (int b = H.level_start[l]; b < H.level_start[l + 1]; ++b) {
      if (H.box_leaf[b] >= 0) {
        zero_box[b] = zero_leaf[H.box_leaf[b]];
      } else {
        uint8_t z = 1;
        for (int q = 0; q < 4; ++q) z &= zero_box[H.box_child0[b] + q];
        zero_box[b] = z;
      }
    }

  // ---- lists 1 and 3 (per leaf), balance check -------------------------
  H.l1_ptr.assign(L + 1, 0);
  H.l3_ptr.assign(L + 1, 0);
  std::vector<std::vector<std::pair<int, int>>> l1(L);
  std::vector<std::vector<std::pair<int, int>>> l3(L);
  for (int leaf = 0; leaf < L; ++leaf) {
    const int b = H.leaf_box[leaf];
    const int l = H.box_level[b], x = H.box_ix[b], y = H.box_iy[b];
    std::vector<int> coarse_seen;
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        const int cx = x + dx, cy = y + dy;
        if (cx < 0 || cy < 0 || cx >= (1 << l) || cy >= (1 << l)) continue;
        const int c = find(l, cx, cy);
        if (c >= 0) {
          if (H.box_leaf[c] >= 0) {
            if (!zero_leaf[H.box_leaf[c]]) l1[leaf].push_back({H.box_leaf[c], (dx + 1) * 3 + (dy + 1)});
          } else {
            for (int q = 0; q < 4; ++q) {
              const int ch = H.box_child0[c] + q;
              const int kx = H.box_ix[ch], ky = H.box_iy[ch];
              if (touch(l, x, y, l + 1, kx, ky)) {
                if (H.box_leaf[ch] < 0) {
                  err = "tree: not level-restricted (leaf " + std::to_string(leaf) +
                        " touches a box two levels finer)";
                  return VFX_ETREE;
                }
                const int ox4 = (2 * kx + 1) - 2 * (2 * x + 1), oy4 = (2 * ky + 1) - 2 * (2 * y + 1);
                if (!zero_leaf[H.box_leaf[ch]])
                  l1[leaf].push_back({H.box_leaf[ch], 21 + near_config_fine_index(ox4, oy4)});
              } else {
                const int ox = (2 * kx + 1) - 2 * (2 * x + 1), oy = (2 * ky + 1) - 2 * (2 * y + 1);
                if (std::max(std::abs(ox), std::abs(oy)) != 5) {
                  err = "internal: bad list-3 configuration";
                  return VFX_EINVAL;
                }
                if (!zero_box[ch]) l3[leaf].push_back({ch, ((ox + 5) / 2) * 6 + (oy + 5) / 2});
              }
            }
          }
        } else {
          const int p = find(l - 1, cx >> 1, cy >> 1);
          if (p < 0 || H.box_leaf[p] < 0) {
            err = "tree: not level-restricted (leaf " + std::to_string(leaf) +
                  " touches a leaf two levels coarser)";
            return VFX_ETREE;
          }
          if (std::find(coarse_seen.begin(), coarse_seen.end(), p) != coarse_seen.end()) continue;
          coarse_seen.push_back(p);
          const int ox2 = (4 * H.box_ix[p] + 2) - (2 * x + 1), oy2 = (4 * H.box_iy[p] + 2) - (2 * y + 1);
          const int ci = near_config_coarse_index(ox2, oy2);
          if (ci < 0) {
            err = "internal: bad coarse configuration";
            return VFX_EINVAL;
          }
          if (!zero_leaf[H.box_leaf[p]]) l1[leaf].push_back({H.box_leaf[p], 9 + ci});
        }
      }
  }
  for (int leaf = 0; leaf < L; ++leaf) {
    H.l1_ptr[leaf + 1] = H.l1_ptr[leaf] + (int)l1[leaf].size();
    for (auto& pr : l1[leaf]) {
      H.l1_src.push_back(pr.first);
      H.l1_cfg.push_back(pr.second);
    }
    H.l3_ptr[leaf + 1] = H.l3_ptr[leaf] + (int)l3[leaf].size();
    for (auto& pr : l3[leaf]) {
      H.l3_src.push_back(pr.first);
      H.l3_cfg.push_back(pr.second);
    }
  }
  // ---- list-1 pairs grouped by configuration -----------------------------
  for (int leaf = 0; leaf < L; ++leaf)
    if (H.l1_ptr[leaf + 1] - H.l1_ptr[leaf] > kNearConfigs) {
      err = "internal: list 1 of a leaf longer than the number of near configurations";
      return VFX_EINVAL;
    }
  H.l1_srcbox.resize(H.l1_src.size());
  for (size_t e = 0; e < H.l1_src.size(); ++e) H.l1_srcbox[e] = H.leaf_box[H.l1_src[e]];
  {
    int rc = build_near_tiles(T, H, 0, 0, err);
    if (rc) return rc;
  }
  // ---- lists 2 and 4 (per box, level >= 2) ------------------------------
  H.l2_ptr.assign(B + 1, 0);
  H.l4_ptr.assign(B + 1, 0);
  for (int b = 0; b < B; ++b) {
    const int l = H.box_level[b];
    int n2 = 0, n4 = 0;
    if (l >= 2) {
      const int x = H.box_ix[b], y = H.box_iy[b];
      const int px = x >> 1, py = y >> 1;
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy) {
          const int c = find(l - 1, px + dx, py + dy);
          if (c < 0) continue;
          if (H.box_leaf[c] < 0) {
            for (int q = 0; q < 4; ++q) {
              const int ch = H.box_child0[c] + q;
              const int kx = H.box_ix[ch], ky = H.box_iy[ch];
              if (touch(l, x, y, l, kx, ky) || zero_box[ch]) continue;
              H.l2_src.push_back(ch);
              H.l2_off.push_back((kx - x + 3) * 7 + (ky - y + 3));
              ++n2;
            }
          } else if (!touch(l, x, y, l - 1, px + dx, py + dy) && !zero_leaf[H.box_leaf[c]]) {
            const int ox2 = (4 * (px + dx) + 2) - (2 * x + 1), oy2 = (4 * (py + dy) + 2) - (2 * y + 1);
            H.l4_src.push_back(H.box_leaf[c]);
            H.l4_cfg.push_back(((ox2 + 5) / 2) * 6 + (oy2 + 5) / 2);
            ++n4;
          }
        }
    }
    H.l2_ptr[b + 1] = H.l2_ptr[b] + n2;
    H.l4_ptr[b + 1] = H.l4_ptr[b] + n4;
  }

  // ---- list-2 target per entry; groups of boxes for the M2L kernel --------
  H.l2_tgt.resize(H.l2_src.size());
  for (int b = 0; b < B; ++b)
    for (int e = H.l2_ptr[b]; e < H.l2_ptr[b + 1]; ++e) H.l2_tgt[e] = b;
  if (H.nlev > 2) {
    int b = H.level_start[2];
    H.m2l_grp.push_back(b);
    while (b < B) {
      int nb = 0, ne = 0;
      while (b < B && nb < 8 && ne + (H.l2_ptr[b + 1] - H.l2_ptr[b]) <= 64) {
        ne += H.l2_ptr[b + 1] - H.l2_ptr[b];
        ++nb;
        ++b;
      }
      if (nb == 0) {
        err = "internal: list 2 longer than 64";
        return VFX_EINVAL;
      }
      H.m2l_grp.push_back(b);
    }
  }
  // ---- upward pass: every non-leaf box at level >= 2 gathers the
  // multipoles of its leaf descendants directly (one translation per
  // (ancestor, leaf) pair, no level-by-level chain).  Pairs are ordered by
  // box, then by leaf box; groups of <= 8 boxes and <= 64 pairs go to one
  // wave, a box with more pairs is split into slices whose partial sums are
  // added in slice order by a second kernel.
  {
    std::vector<int> pos(B, -1);
    for (int b = H.level_start[std::min(2, H.nlev)]; b < B; ++b)
      if (H.box_leaf[b] < 0) {
        pos[b] = (int)H.up_box.size();
        H.up_box.push_back(b);
      }
    const int nU = (int)H.up_box.size();
    std::vector<std::vector<int>> lst(nU);
    for (int b = 0; b < B; ++b) {
      // a leaf whose data vanish identically adds nothing to any multipole
      if (H.box_leaf[b] < 0 || zero_leaf[H.box_leaf[b]]) continue;
      for (int a = H.box_parent[b]; a >= 0 && H.box_level[a] >= 2; a = H.box_parent[a]) lst[pos[a]].push_back(b);
    }
    H.up_ptr.assign(nU + 1, 0);
    for (int u = 0; u < nU; ++u) {
      std::sort(lst[u].begin(), lst[u].end());
      H.up_ptr[u + 1] = H.up_ptr[u] + (int)lst[u].size();
      for (int b : lst[u]) {
        H.up_src.push_back(b);
        H.up_pos.push_back(u);
      }
    }
    int u = 0, slots = 0;
    while (u < nU) {
      const int cnt = H.up_ptr[u + 1] - H.up_ptr[u];
      if (cnt > 64) {
        const int ns = (cnt + 63) / 64;
        H.up_split.insert(H.up_split.end(), {H.up_box[u], slots, ns});
        for (int j = 0; j < ns; ++j) {
          const int e0 = H.up_ptr[u] + 64 * j;
          H.up_grp.insert(H.up_grp.end(), {u, u + 1, e0, std::min(e0 + 64, H.up_ptr[u + 1]), slots++});
        }
        ++u;
        continue;
      }
      int v = u, ne = 0;
      while (v < nU && v - u < 8 && ne + (H.up_ptr[v + 1] - H.up_ptr[v]) <= 64) {
        ne += H.up_ptr[v + 1] - H.up_ptr[v];
        ++v;
      }
      H.up_grp.insert(H.up_grp.end(), {u, v, H.up_ptr[u], H.up_ptr[v], -1});
      u = v;
    }
    H.up_slots = slots;
    // downward pass: (leaf, ancestor at level >= 2) pairs, nearest ancestor
    // first, and wave groups of <= 8 leaves with <= 64 pairs
    H.anc_ptr.assign(L + 1, 0);
    for (int leaf = 0; leaf < L; ++leaf) {
      for (int a = H.box_parent[H.leaf_box[leaf]]; a >= 0 && H.box_level[a] >= 2; a = H.box_parent[a]) {
        H.anc.push_back(a);
        H.anc_leaf.push_back(leaf);
      }
      H.anc_ptr[leaf + 1] = (int)H.anc.size();
    }
    int f = 0;
    H.dn_grp.push_back(0);
    while (f < L) {
      int g = f;
      while (g < L && g - f < 8 && H.anc_ptr[g + 1] - H.anc_ptr[f] <= 64) ++g;
      if (g == f) {
        err = "internal: more than 64 ancestors";
        return VFX_EINVAL;
      }
      H.dn_grp.push_back(g);
      f = g;
    }
  }
  // ---- list-4 entries grouped by P2L slot --------------------------------
  {
    const int N4 = H.l4_ptr[B];
    std::vector<int> cnt(kP2LSlots + 1, 0);
    for (int e = 0; e < N4; ++e) cnt[H.l4_cfg[e] + 1]++;
    for (int c = 0; c < kP2LSlots; ++c) cnt[c + 1] += cnt[c];
    H.p4_src.assign(N4, 0);
    H.l4_slot.assign(N4, 0);
    std::vector<int> pos(cnt.begin(), cnt.end() - 1);
    for (int b = 0; b < B; ++b)
      for (int e = H.l4_ptr[b]; e < H.l4_ptr[b + 1]; ++e) {
        const int s = pos[H.l4_cfg[e]]++;
        H.p4_src[s] = H.l4_src[e];
        H.l4_slot[e] = s;
      }
    for (int c = 0; c < kP2LSlots; ++c)
      for (int f = cnt[c]; f < cnt[c + 1]; f += 64) {
        H.t4_cfg.push_back(c);
        H.t4_first.push_back(f);
        H.t4_count.push_back(std::min(64, cnt[c + 1] - f));
      }
  }
  // ---- list-3 entries grouped by M2P slot --------------------------------
  {
    const int N3 = H.l3_ptr[L];
    std::vector<int> cnt(kP2LSlots + 1, 0);
    for (int e = 0; e < N3; ++e) cnt[H.l3_cfg[e] + 1]++;
    for (int c = 0; c < kP2LSlots; ++c) cnt[c + 1] += cnt[c];
    H.p3_src.assign(N3, 0);
    H.l3_slot.assign(N3, 0);
    std::vector<int> pos(cnt.begin(), cnt.end() - 1);
    for (int e = 0; e < N3; ++e) {
      const int s = pos[H.l3_cfg[e]]++;
      H.p3_src[s] = H.l3_src[e];
      H.l3_slot[e] = s;
    }
    for (int c = 0; c < kP2LSlots; ++c)
      for (int f = cnt[c]; f < cnt[c + 1]; f += 64) {
        H.t3_cfg.push_back(c);
        H.t3_first.push_back(f);
        H.t3_count.push_back(std::min(64, cnt[c + 1] - f));
      }
  }
  // P2M: every leaf with possibly nonzero data, one configuration
  // (a leaf whose data vanish identically is no source of anything, so its
  // multipole is neither formed nor read)
  H.leaf_ids.clear();
  for (int i = 0; i < L; ++i)
    if (!zero_leaf[i]) H.leaf_ids.push_back(i);
  const int NL0 = (int)H.leaf_ids.size();
  for (int f = 0; f < NL0; f += 64) {
    H.t0_cfg.push_back(0);
    H.t0_first.push_back(f);
    H.t0_count.push_back(std::min(64, NL0 - f));
  }

  // ---- per-cut-leaf pseudo-inverses --------------------------------------
  const int nX = T.nX, nG = T.nG, Kb2 = T.Kbar * T.Kbar;
  if (H.ncut > 0 && !tree->cut_mask) {
    err = "tree: cut leaves present but no cut_mask";
    return VFX_EINVAL;
  }
  H.pinv_ptr.assign(H.ncut + 1, 0);
  H.sbar_given.assign((size_t)H.ncut * Kb2, 0);
  for (int c = 0; c < H.ncut; ++c) {
    const uint8_t* m = tree->cut_mask + (size_t)c * nX;
    int ni = 0;
    for (int k = 0; k < nX; ++k) ni += m[k] ? 1 : 0;
    H.pinv_ptr[c + 1] = H.pinv_ptr[c] + ni;
    for (int a = 0; a < Kb2; ++a) H.sbar_given[(size_t)c * Kb2 + a] = m[T.n + a] ? 1 : 0;
  }
  H.pinv_idx.resize(H.pinv_ptr[H.ncut]);
  H.factored = !defer_factor;
  if (H.factored) H.pinv_val.assign((size_t)H.pinv_ptr[H.ncut] * nG, 0.0);
  for (int c = 0; c < H.ncut; ++c) {
    const uint8_t* m = tree->cut_mask + (size_t)c * nX;
    int q = H.pinv_ptr[c];
    for (int k = 0; k < nX; ++k)
      if (m[k]) H.pinv_idx[q++] = (uint16_t)k;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < (H.factored ? H.ncut : 0); ++c) {
    const int off = H.pinv_ptr[c], ni = H.pinv_ptr[c + 1] - off;
    if (ni == 0) continue;
    std::vector<double> AI((size_t)ni * nG);
    for (int r = 0; r < ni; ++r)
      std::memcpy(&AI[(size_t)r * nG], &T.A[(size_t)H.pinv_idx[off + r] * nG], sizeof(double) * nG);
    // P (nG x ni) stored row-major at pinv_val + off*nG
    pinv_jacobi(AI.data(), ni, nG, 1e-13, &H.pinv_val[(size_t)off * nG]);
  }
  H.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return VFX_OK;
}

}  // namespace vfx
