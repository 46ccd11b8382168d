// Nested-dissection plan of the coarse saddle point (host side).
//
// The coarse unknowns of Algorithm "BDDC preconditioner" step 1 are the face
// averages and adaptive rows of every face (Section 4) and one rescaled
// pressure per subdomain (the last subdomain's pressure is pinned).  A
// subdomain's coarse dofs form a dense clique of the coarse matrix, and two
// subdomains couple only through the dofs of a face they share, so the
// subdomain grid dissects like a Cartesian mesh: a plane of faces splits a box
// of subdomains into two boxes that do not couple.  Recursive bisection of the
// box along its longest axis gives a tree of separator fronts; a leaf box (at
// most `leaf` subdomains) keeps its interior faces as one front.
//
// A pressure joins the front of the separator nearest the root among those
// that hold one of its faces, so it is eliminated after every face it couples
// to.  Then each leading principal block of the coarse matrix is a saddle
// point with an SPD flux block and divergence rows of full rank, so the signed
// factorization K = L diag(s) L^T exists with s = +1 on face dofs and -1 on
// pressures, without pivoting.
//
// Fronts are numbered level by level (height above the leaves, then creation
// order) and the coarse dofs follow the front order, so the fronts of one
// level, their dofs and their work vectors are contiguous.  For front p with
// own dofs P (n_p) and later dofs B(p) (m_p) it couples to after elimination
// (the boundary of its subtree, all in ancestor fronts), the plan records
// B(p), the position of every entry of B(p) in the parent's index list
// [P(parent), B(parent)] (extend-add map) and the storage offsets.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <stdexcept>
#include <vector>

#include "layout.hpp"

namespace bddc {

struct NdPlan {
  int H = 0;                        // levels
  int nfr = 0;                      // fronts
  int nk = 0;                       // coarse dofs (pinned pressure excluded)
  std::vector<int> lvl_off;         // [H+1] fronts of level h
  std::vector<int> lvl_dof;         // [H+1] coarse dofs of level h
  std::vector<int> first, n, m;     // per front: first own dof, own dofs, later dofs
  std::vector<int> ch;              // [2 nfr] children (-1: none)
  std::vector<int> b_off, bidx;     // [nfr+1], B(p) ascending
  std::vector<int> ext;             // aligned with bidx: position in the parent's list
  std::vector<int> touch_off, touch;  // subdomains whose coarse dofs meet front p
  std::vector<int> face_cofs;       // per face: its first coarse dof
  std::vector<int> pidx;            // per subdomain: pressure dof or -1
  std::vector<int> dfront;          // [nk] front of every dof
  std::vector<int64_t> F_off, w_off, q_off, r_off, v_off;  // [nfr+1] storage prefix sums
  // solve sweeps (coarse.hip): lane-group width per front, the slot (0/1) of
  // every front among its parent's children, forward push targets of the B
  // rows, backward scatter targets of the own dofs and the copies of the
  // parents' B values into their children's B vectors
  std::vector<int> gf, gb;          // [nfr] group widths, forward rows / backward columns
  std::vector<int> parent;          // [nfr] parent front (-1: root)
  int wide1 = 0, wide4 = 24, wide16 = 96;  // rows (columns) up to wide1 long take 1 lane, up to wide4 4,
                                           // up to wide16 16, longer ones 64
  std::vector<int> cslot;           // [nfr]
  std::vector<int> wdst;            // [sum m] forward: position of w_c[k] in the parent's vectors
  std::vector<int> xsc_off, xsc;    // [nk+1], [sum m]: every B-vector position holding x[d]
  // task descriptors (four int4 each, see coarse.hip): all forward tasks by
  // ascending level, then all backward tasks by descending level
  std::vector<int> task;            // [16 ntask]
  int ntask = 0;
  std::vector<int> ftask_off;       // [H+1] forward tasks of level h
  std::vector<int> btask_lo, btask_hi;  // [H] backward tasks of level h
  std::vector<int> ft_first, bt_first;  // [nfr] first forward / backward task of each front
  std::vector<int> lvl_maxn, lvl_maxnm;  // [H] largest n_p and n_p + m_p of the level's fronts
  // bottom subtrees (nd_subtrees): the fronts of levels [0, sub_lv] are swept
  // in one launch per direction, one workgroup per subtree (a front of level
  // <= sub_lv whose parent lies above sub_lv, with all its descendants) taking
  // the subtree's levels one after the other.  stask holds copies of the
  // subtrees' forward tasks, then of their backward tasks; subtree t's phase k
  // (k = 0 .. sub_lv) is stask[sph[t (sub_lv + 2) + k], sph[t (sub_lv + 2) + k + 1])
  // forward (level k), and the same at sph[nsubt (sub_lv + 2) + t (sub_lv + 2) + k]
  // backward (level sub_lv - k).
  int sub_lv = -1;                  // -1: every level has its own launches
  int nsubt = 0;
  std::vector<int> stask, sph;
  // dense top block (nd_dense_top): levels [top, H) are solved with the
  // explicit inverse of their Schur complement; their nt dofs are the last
  // ones, [lvl_dof[top], nk).  tg lists, for every top dof, the positions of
  // the top fronts' work vectors (own part and B part) that hold updates of it.
  int top = 0;                      // H: no dense block
  int nt = 0;
  std::vector<int> tg_off, tg;      // [nt+1], positions
};

inline void nd_subtrees(NdPlan &P, int lv);

// Lane-group widths and the task list of the solve sweeps.  A row (forward)
// or column (backward) of at most wide1 entries is handled by one lane, of at
// most wide4 by 4 lanes, of at most wide16 by 16, longer ones by 64 (wide1 = 0:
// no single-lane class), so that short rows do not leave lanes
// idle; a workgroup of 256 lanes takes 256 / g of them.  Called by nd_plan
// with the defaults and again by the autotuner with other thresholds (the
// factor and the dense top block do not depend on them).
inline void nd_tasks(NdPlan &P, int wide4, int wide16, int wide1 = -1) {
  const int nn = P.nfr, H = P.H;
  if (wide1 >= 0) P.wide1 = wide1;   // < 0: keep
  P.wide4 = wide4;
  P.wide16 = wide16;
  const int w1 = P.wide1;
  auto width = [&](int len) { return len <= w1 ? 1 : (len <= wide4 ? 4 : (len <= wide16 ? 16 : 64)); };
  P.gf.assign(nn, 4);
  P.gb.assign(nn, 4);
  for (int r = 0; r < nn; ++r) {
    P.gf[r] = width(P.n[r]);
    P.gb[r] = width(P.n[r] + P.m[r]);
  }
  P.task.clear();
  // Task descriptors, four int4 each:
  //   {front, first row / column, lane-group width, n}, {m, first dof, v_off, b_off},
  //   {r_off low 32 bits, r_off high 32 bits, child slot, kind (0 forward, 1 backward)},
  //   {dependency a, count a, dependency b, count b}  (-1: none)
  // One workgroup (256 lanes) takes 256/g rows (forward) or columns (backward).
  // The dependencies name what a task reads (p: the forward tasks of front p,
  // nfr + p: its backward tasks, with their number): a forward task reads its
  // children's forward results, a backward task its parent's backward results
  // (the root: its own forward results).  The list is in topological order;
  // the host plan test checks both against the level order of the sweeps.
  std::vector<int> nft(nn, 0), nbt(nn, 0);
  for (int r = 0; r < nn; ++r) {
    const int fr = 256 / P.gf[r], br = 256 / P.gb[r];
    nft[r] = (P.n[r] + P.m[r] + fr - 1) / fr;
    nbt[r] = (P.n[r] + br - 1) / br;
  }
  auto push = [&](int r, int j, int g, int kind) {
    const int64_t ro = P.r_off[r];
    int da = -1, ta = 0, db = -1, tb = 0;
    if (kind == 0) {
      const int c0 = P.ch[2 * r], c1 = P.ch[2 * r + 1];
      if (c0 >= 0) { da = c0; ta = nft[c0]; }
      if (c1 >= 0) { db = c1; tb = nft[c1]; }
    } else if (P.parent[r] >= 0) {
      da = nn + P.parent[r];
      ta = nbt[P.parent[r]];
    } else {
      da = r;
      ta = nft[r];
    }
    const int d[16] = {r, j, g, P.n[r], P.m[r], P.first[r], (int)P.v_off[r], P.b_off[r],
                       (int)(uint32_t)(ro & 0xffffffff), (int)(uint32_t)(ro >> 32), P.cslot[r], kind,
                       da, ta, db, tb};
    P.task.insert(P.task.end(), d, d + 16);
  };
  P.ftask_off.assign(H + 1, 0);
  P.btask_lo.assign(H, 0);
  P.btask_hi.assign(H, 0);
  P.lvl_maxn.assign(H, 0);
  P.lvl_maxnm.assign(H, 0);
  for (int h = 0; h < H; ++h)
    for (int r = P.lvl_off[h]; r < P.lvl_off[h + 1]; ++r) {
      P.lvl_maxn[h] = std::max(P.lvl_maxn[h], P.n[r]);
      P.lvl_maxnm[h] = std::max(P.lvl_maxnm[h], P.n[r] + P.m[r]);
    }
  P.ft_first.assign(nn, 0);
  P.bt_first.assign(nn, 0);
  for (int h = 0; h < H; ++h) {
    for (int r = P.lvl_off[h]; r < P.lvl_off[h + 1]; ++r) {
      P.ft_first[r] = (int)P.task.size() / 16;
      for (int j = 0; j < P.n[r] + P.m[r]; j += 256 / P.gf[r]) push(r, j, P.gf[r], 0);
    }
    P.ftask_off[h + 1] = (int)P.task.size() / 16;
  }
  for (int h = H - 1; h >= 0; --h) {
    P.btask_lo[h] = (int)P.task.size() / 16;
    for (int r = P.lvl_off[h]; r < P.lvl_off[h + 1]; ++r) {
      P.bt_first[r] = (int)P.task.size() / 16;
      for (int j = 0; j < P.n[r]; j += 256 / P.gb[r]) push(r, j, P.gb[r], 1);
    }
    P.btask_hi[h] = (int)P.task.size() / 16;
  }
  P.ntask = (int)P.task.size() / 16;
  nd_subtrees(P, P.sub_lv);   // the subtree lists copy the tasks just built
}

// Bottom subtrees of the sweeps: levels [0, lv] (at most the levels below the
// dense top block) in one launch per direction.  Inside a subtree a front's
// forward pushes go to its parent, which is in the subtree unless the front is
// its root (then the parent is swept by a later launch), and its backward
// values go to the B vectors of its descendants; so subtrees never read what
// another one writes in the same launch.  Subtrees are listed largest first.
// Call after nd_tasks and nd_dense_top; lv < 0 clears the subtree lists.
inline void nd_subtrees(NdPlan &P, int lv) {
  P.sub_lv = -1;
  P.nsubt = 0;
  P.stask.clear();
  P.sph.clear();
  lv = std::min(lv, P.top - 1);
  if (lv < 0 || P.nfr == 0) return;
  const int nn = P.nfr;
  std::vector<int> level(nn, 0);
  for (int h = 0; h < P.H; ++h)
    for (int r = P.lvl_off[h]; r < P.lvl_off[h + 1]; ++r) level[r] = h;
  auto ntask = [&](int r, int kind) {
    const int per = 256 / (kind == 0 ? P.gf[r] : P.gb[r]);
    return ((kind == 0 ? P.n[r] + P.m[r] : P.n[r]) + per - 1) / per;
  };
  // subtrees: fronts of each root by level; size = forward tasks
  std::vector<std::vector<std::vector<int>>> sub;
  std::vector<int64_t> size;
  for (int r = 0; r < P.lvl_off[lv + 1]; ++r) {
    const int p = P.parent[r];
    if (p >= 0 && level[p] <= lv) continue;
    std::vector<std::vector<int>> byl(lv + 1);
    std::vector<int> stack{r};
    int64_t sz = 0;
    while (!stack.empty()) {
      const int q = stack.back();
      stack.pop_back();
      byl[level[q]].push_back(q);
      sz += ntask(q, 0);
      for (int k = 0; k < 2; ++k)
        if (P.ch[2 * q + k] >= 0) stack.push_back(P.ch[2 * q + k]);
    }
    for (auto &v : byl) std::sort(v.begin(), v.end());
    sub.push_back(std::move(byl));
    size.push_back(sz);
  }
  std::vector<int> order(sub.size());
  for (size_t t = 0; t < order.size(); ++t) order[t] = (int)t;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return size[a] > size[b]; });
  const int nt = (int)sub.size(), np = lv + 2;
  P.sub_lv = lv;
  P.nsubt = nt;
  P.sph.assign(2 * (size_t)nt * np, 0);
  auto copy = [&](int r, int kind) {
    const int t0 = kind == 0 ? P.ft_first[r] : P.bt_first[r];
    P.stask.insert(P.stask.end(), P.task.begin() + 16 * (int64_t)t0,
                   P.task.begin() + 16 * (int64_t)(t0 + ntask(r, kind)));
  };
  for (int kind = 0; kind < 2; ++kind)
    for (int t = 0; t < nt; ++t) {
      int *ph = &P.sph[(size_t)kind * nt * np + (size_t)t * np];
      for (int k = 0; k <= lv; ++k) {
        ph[k] = (int)P.stask.size() / 16;
        for (int r : sub[order[t]][kind == 0 ? k : lv - k]) copy(r, kind);
      }
      ph[lv + 1] = (int)P.stask.size() / 16;
    }
}

// `leaf`: largest number of subdomains in a leaf box (>= 1).
inline void nd_plan(const Layout &L, const std::vector<int> &face_k, int leaf, NdPlan &P) {
  const int N = L.N, nF = L.nF;
  if (leaf < 1) leaf = 1;
  struct Node {
    int lo[3], hi[3];
    int ch[2] = {-1, -1};
    int depth = 0, height = 0;
    std::vector<int> faces, press;
  };
  std::vector<Node> nodes;
  std::vector<int> face_node(nF, -1);
  std::vector<int> fpos(3 * nF);   // subdomain-grid position of every face's minus side
  for (int f = 0; f < nF; ++f)
    for (int e = 0; e < 3; ++e) fpos[3 * f + e] = (L.f_minus[f] / L.sstride[e]) % L.nsub[e];
  // faces of a box interior, or of its cut plane (axis d, between layers cut-1 and cut)
  auto collect = [&](const int *lo, const int *hi, int d, int cut, std::vector<int> &out) {
    for (int f = 0; f < nF; ++f) {
      const int *s = &fpos[3 * f];
      bool in = true;
      for (int e = 0; e < 3; ++e) in = in && s[e] >= lo[e] && s[e] < hi[e];
      if (!in) continue;
      const int fd = L.f_dir[f];
      if (s[fd] + 1 >= hi[fd]) continue;      // the plus side lies outside the box
      if (d >= 0 && (fd != d || s[d] != cut - 1)) continue;
      out.push_back(f);
    }
  };
  // coarse dofs of the +d face of every subdomain (0 where there is none)
  std::vector<int> wface(3 * (size_t)N, 0);
  for (int f = 0; f < nF; ++f) wface[3 * (size_t)L.f_minus[f] + L.f_dir[f]] = 1 + face_k[f];
  // dofs of the plane between layers cut-1 and cut (axis d) inside the box
  auto plane_weight = [&](const int *lo, const int *hi, int d, int cut) {
    const int a = (d + 1) % 3, b = (d + 2) % 3;
    int64_t w = 0;
    int s[3];
    s[d] = cut - 1;
    for (s[a] = lo[a]; s[a] < hi[a]; ++s[a])
      for (s[b] = lo[b]; s[b] < hi[b]; ++s[b])
        w += wface[3 * (size_t)(s[0] * L.sstride[0] + s[1] * L.sstride[1] + s[2] * L.sstride[2]) + d];
    return w;
  };
  // recursive bisection; returns the node id or -1 (box without faces).  The
  // cut is the plane with the fewest coarse dofs among those that leave at
  // least a quarter of the box extent on either side (ties: the more balanced
  // cut, then the lower axis), so that faces rich in adaptive constraints end
  // up in small fronts low in the tree.
  auto build = [&](auto &&self, const int *lo, const int *hi, int depth) -> int {
    int ext[3], cnt = 1;
    for (int e = 0; e < 3; ++e) {
      ext[e] = hi[e] - lo[e];
      cnt *= ext[e];
    }
    Node nd;
    for (int e = 0; e < 3; ++e) { nd.lo[e] = lo[e]; nd.hi[e] = hi[e]; }
    nd.depth = depth;
    if (cnt <= leaf) {
      collect(lo, hi, -1, 0, nd.faces);
      if (nd.faces.empty()) return -1;
      nodes.push_back(nd);
      return (int)nodes.size() - 1;
    }
    int d = -1, cut = 0;
    int64_t bw = 0;
    int bimb = 0;
    for (int e = 0; e < 3; ++e) {
      if (ext[e] < 2) continue;
      const int side = std::max(1, (ext[e] + 3) / 4);
      for (int c = lo[e] + side; c <= hi[e] - side; ++c) {
        const int64_t w = plane_weight(lo, hi, e, c);
        const int imb = std::abs((c - lo[e]) - (hi[e] - c));
        if (d < 0 || w < bw || (w == bw && imb < bimb)) {
          d = e;
          cut = c;
          bw = w;
          bimb = imb;
        }
      }
    }
    int hi1[3] = {hi[0], hi[1], hi[2]}, lo2[3] = {lo[0], lo[1], lo[2]};
    hi1[d] = cut;
    lo2[d] = cut;
    const int c0 = self(self, lo, hi1, depth + 1);
    const int c1 = self(self, lo2, hi, depth + 1);
    collect(lo, hi, d, cut, nd.faces);
    nd.ch[0] = c0;
    nd.ch[1] = c1;
    nodes.push_back(nd);
    return (int)nodes.size() - 1;
  };
  const int lo0[3] = {0, 0, 0}, hi0[3] = {L.nsub[0], L.nsub[1], L.nsub[2]};
  if (N > 1) build(build, lo0, hi0, 0);
  const int nn = (int)nodes.size();
  for (int q = 0; q < nn; ++q)
    for (int f : nodes[q].faces) {
      if (face_node[f] >= 0) throw std::logic_error("coarse plan: face in two fronts");
      face_node[f] = q;
    }
  for (int f = 0; f < nF; ++f)
    if (face_node[f] < 0) throw std::logic_error("coarse plan: face in no front");
  // pressures: the front nearest the root among those holding a face of i
  for (int i = 0; i + 1 < N; ++i) {
    int best = -1;
    for (int t = L.sub_face_off[i]; t < L.sub_face_off[i + 1]; ++t) {
      const int q = face_node[L.sub_faces[t]];
      if (best < 0 || nodes[q].depth < nodes[best].depth) best = q;
    }
    if (best < 0) throw std::logic_error("coarse plan: subdomain without faces");
    nodes[best].press.push_back(i);
  }
  // heights (children are created before their parent)
  for (int q = 0; q < nn; ++q) {
    int hq = 0;
    for (int c : nodes[q].ch)
      if (c >= 0) hq = std::max(hq, nodes[c].height + 1);
    nodes[q].height = hq;
  }
  int H = 0;
  for (int q = 0; q < nn; ++q) H = std::max(H, nodes[q].height + 1);
  std::vector<int> order(nn);
  for (int q = 0; q < nn; ++q) order[q] = q;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return nodes[a].height < nodes[b].height; });
  std::vector<int> fid(nn);
  for (int r = 0; r < nn; ++r) fid[order[r]] = r;

  P = NdPlan();
  P.H = H;
  P.nfr = nn;
  P.lvl_off.assign(H + 1, 0);
  P.lvl_dof.assign(H + 1, 0);
  P.first.assign(nn, 0);
  P.n.assign(nn, 0);
  P.m.assign(nn, 0);
  P.ch.assign(2 * nn, -1);
  P.face_cofs.assign(nF, -1);
  P.pidx.assign(N, -1);
  int cur = 0;
  for (int r = 0; r < nn; ++r) {
    Node &nd = nodes[order[r]];
    std::sort(nd.faces.begin(), nd.faces.end());
    std::sort(nd.press.begin(), nd.press.end());
    P.first[r] = cur;
    for (int f : nd.faces) {
      P.face_cofs[f] = cur;
      cur += 1 + face_k[f];
    }
    for (int i : nd.press) P.pidx[i] = cur++;
    P.n[r] = cur - P.first[r];
    for (int k = 0; k < 2; ++k) P.ch[2 * r + k] = nd.ch[k] >= 0 ? fid[nd.ch[k]] : -1;
    if (P.ch[2 * r] < 0 && P.ch[2 * r + 1] >= 0) std::swap(P.ch[2 * r], P.ch[2 * r + 1]);
  }
  P.nk = cur;
  for (int h = 0, r = 0; h <= H; ++h) {
    while (r < nn && nodes[order[r]].height < h) ++r;
    P.lvl_off[h] = r;
    P.lvl_dof[h] = r < nn ? P.first[r] : cur;
  }
  P.dfront.assign(cur, 0);
  for (int r = 0; r < nn; ++r)
    for (int k = 0; k < P.n[r]; ++k) P.dfront[P.first[r] + k] = r;
  // coarse dofs of every subdomain, and the subdomains meeting every front
  std::vector<std::vector<int>> D(N);
  std::vector<std::vector<int>> tch(nn);
  for (int i = 0; i < N; ++i) {
    for (int t = L.sub_face_off[i]; t < L.sub_face_off[i + 1]; ++t) {
      const int f = L.sub_faces[t];
      for (int l = 0; l <= face_k[f]; ++l) D[i].push_back(P.face_cofs[f] + l);
      tch[fid[face_node[f]]].push_back(i);
    }
    if (P.pidx[i] >= 0) {
      D[i].push_back(P.pidx[i]);
      tch[P.dfront[P.pidx[i]]].push_back(i);
    }
    std::sort(D[i].begin(), D[i].end());
  }
  P.touch_off.assign(nn + 1, 0);
  for (int r = 0; r < nn; ++r) {
    std::sort(tch[r].begin(), tch[r].end());
    tch[r].erase(std::unique(tch[r].begin(), tch[r].end()), tch[r].end());
    P.touch_off[r + 1] = P.touch_off[r] + (int)tch[r].size();
    P.touch.insert(P.touch.end(), tch[r].begin(), tch[r].end());
  }
  // B(p) = (coarse dofs of the touching subdomains and children's B) beyond p
  std::vector<std::vector<int>> Bs(nn);
  for (int r = 0; r < nn; ++r) {
    const int last = P.first[r] + P.n[r] - 1;
    std::vector<int> s;
    for (int i : tch[r])
      for (int v : D[i])
        if (v > last) s.push_back(v);
    for (int k = 0; k < 2; ++k) {
      const int c = P.ch[2 * r + k];
      if (c < 0) continue;
      for (int v : Bs[c]) {
        if (v < P.first[r]) throw std::logic_error("coarse plan: child couples outside its ancestors");
        if (v > last) s.push_back(v);
      }
    }
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    Bs[r] = s;
    P.m[r] = (int)s.size();
  }
  P.b_off.assign(nn + 1, 0);
  for (int r = 0; r < nn; ++r) P.b_off[r + 1] = P.b_off[r] + P.m[r];
  P.bidx.reserve(P.b_off[nn]);
  for (int r = 0; r < nn; ++r) P.bidx.insert(P.bidx.end(), Bs[r].begin(), Bs[r].end());
  // extend-add maps: position of B(c)[k] in [own(p), B(p)]
  P.ext.assign(P.b_off[nn], -1);
  std::vector<int> parent(nn, -1);
  for (int r = 0; r < nn; ++r)
    for (int k = 0; k < 2; ++k)
      if (P.ch[2 * r + k] >= 0) parent[P.ch[2 * r + k]] = r;
  for (int c = 0; c < nn; ++c) {
    const int p = parent[c];
    if (p < 0) {
      if (P.m[c] != 0) throw std::logic_error("coarse plan: root with later dofs");
      continue;
    }
    for (int k = 0; k < P.m[c]; ++k) {
      const int v = Bs[c][k];
      int pos;
      if (v < P.first[p] + P.n[p]) {
        pos = v - P.first[p];
      } else {
        auto it = std::lower_bound(Bs[p].begin(), Bs[p].end(), v);
        if (it == Bs[p].end() || *it != v) throw std::logic_error("coarse plan: extend-add map");
        pos = P.n[p] + (int)(it - Bs[p].begin());
      }
      P.ext[P.b_off[c] + k] = pos;
    }
  }
  // storage offsets
  P.F_off.assign(nn + 1, 0);
  P.w_off.assign(nn + 1, 0);
  P.q_off.assign(nn + 1, 0);
  P.r_off.assign(nn + 1, 0);
  P.v_off.assign(nn + 1, 0);
  for (int r = 0; r < nn; ++r) {
    const int64_t a = P.n[r], b = P.m[r];
    P.F_off[r + 1] = P.F_off[r] + (a + b) * (a + b);
    P.w_off[r + 1] = P.w_off[r] + a * a;
    P.q_off[r + 1] = P.q_off[r] + a * b;
    P.r_off[r + 1] = P.r_off[r] + a * (a + 1) / 2 + a * b;
    P.v_off[r + 1] = P.v_off[r] + a + b;
  }
  // sweep maps
  const int64_t nv = P.v_off[nn];
  P.cslot.assign(nn, 0);
  for (int r = 0; r < nn; ++r)
    for (int k = 0; k < 2; ++k)
      if (P.ch[2 * r + k] >= 0) P.cslot[P.ch[2 * r + k]] = k;
  P.parent = parent;
  P.wdst.assign(P.b_off[nn], -1);
  for (int c = 0; c < nn; ++c) {
    const int p = parent[c];
    if (p < 0) continue;
    for (int t = 0; t < P.m[c]; ++t) P.wdst[P.b_off[c] + t] = (int)(P.v_off[p] + P.ext[P.b_off[c] + t]);
  }
  // x[d] goes to every B vector that holds d (the fronts below d's front)
  P.xsc_off.assign(cur + 1, 0);
  for (int v : P.bidx) ++P.xsc_off[v + 1];
  for (int d = 0; d < cur; ++d) P.xsc_off[d + 1] += P.xsc_off[d];
  P.xsc.assign(P.bidx.size(), -1);
  {
    std::vector<int> fillp(P.xsc_off.begin(), P.xsc_off.end() - 1);
    for (int q = 0; q < (int)P.bidx.size(); ++q) P.xsc[fillp[P.bidx[q]]++] = q;
  }
  nd_tasks(P, P.wide4, P.wide16);
  P.top = H;
  P.tg_off.assign(1, 0);
  if (nv > INT32_MAX) throw std::length_error("coarse plan: front vectors too long");
}

// Dense top block.  After the forward sweep of the levels below `top`, the
// dofs of levels top.. H-1 satisfy S_t x_t = t_t, where S_t is the Schur
// complement of the coarse matrix on them and t_t[d] is the right-hand side at
// d plus every update the lower fronts pushed into the top fronts' vectors for
// d (own rows of d's front, B rows of the top fronts below it).  S_t^{-1} is
// formed at setup; a solve then needs one gather and one dense product in
// place of the 2 (H - top) sweep launches of those levels.  `top` is the
// lowest level at which the top block holds at most max_dofs dofs; max_dofs
// <= 0 leaves the plan without a dense block.
inline void nd_dense_top(NdPlan &P, int max_dofs) {
  P.top = P.H;
  P.nt = 0;
  P.tg_off.assign(1, 0);
  P.tg.clear();
  if (max_dofs <= 0 || P.nk == 0) return;
  int top = P.H;
  while (top > 0 && P.nk - P.lvl_dof[top - 1] <= max_dofs) --top;
  if (top == P.H) return;
  const int d0 = P.lvl_dof[top];
  P.top = top;
  P.nt = P.nk - d0;
  std::vector<std::vector<int>> pos(P.nt);
  for (int r = P.lvl_off[top]; r < P.nfr; ++r) {
    for (int k = 0; k < P.n[r]; ++k) pos[P.first[r] + k - d0].push_back((int)P.v_off[r] + k);
    for (int k = 0; k < P.m[r]; ++k) {
      const int v = P.bidx[P.b_off[r] + k];
      if (v < d0) throw std::logic_error("coarse plan: top front couples below the top block");
      pos[v - d0].push_back((int)(P.v_off[r] + P.n[r] + k));
    }
  }
  P.tg_off.assign(P.nt + 1, 0);
  for (int j = 0; j < P.nt; ++j) {
    P.tg_off[j + 1] = P.tg_off[j] + (int)pos[j].size();
    P.tg.insert(P.tg.end(), pos[j].begin(), pos[j].end());
  }
}

}  // namespace bddc
