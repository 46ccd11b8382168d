// Host-side index maps of a box-partitioned Cartesian grid.
//
// Everything here is integer bookkeeping computed once in setup: subdomain
// boxes, local cell numbering, the interface (every interface flux dof is
// shared by exactly two subdomains; RT0 has faces only, no corners or edges,
// Section 3), the faces (pairs of adjacent subdomains) and the
// face-major local ordering of each subdomain's interface dofs.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <stdexcept>
#include <string>
#include <vector>

namespace bddc {

struct Layout {
  int dim = 0;
  int n[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  int64_t ncells = 0, nfaces_all = 0;
  int64_t face_off[4] = {0, 0, 0, 0};
  int fshape[3][3] = {{1, 1, 1}, {1, 1, 1}, {1, 1, 1}};
  int nsub[3] = {1, 1, 1};
  std::vector<int> cuts[3];
  int N = 0;
  int sstride[3] = {1, 1, 1};

  // per subdomain
  std::vector<int> lo[3], ext[3];      // box origin and extent (cells)
  std::vector<int> nc, nG, nI;         // cells, interface dofs, interior faces
  std::vector<int64_t> cell_off, g_off;  // prefix sums
  std::vector<int> lcell_global;       // [sum nc] local cell -> global cell
  // local interface dofs [sum nG]
  std::vector<int> Rmap;               // -> interface index
  std::vector<int> lg_dir, lg_cell, lg_end;  // line-end description (end 0: -d face, 1: +d face)
  std::vector<int> lg_partner;         // local index of the other end of the same line, or -1
  // interface [n_gamma]
  int nGamma = 0;
  std::vector<int64_t> gamma_face;     // global face id (sorted)
  std::vector<int> own_minus, own_plus;  // flat local index in the minus / plus subdomain
  std::vector<int> sub_minus, sub_plus;
  // faces [nF] (pairs of adjacent subdomains, sorted by (minus, plus))
  int nF = 0;
  std::vector<int> f_minus, f_plus, f_n, f_dir, f_loff_minus, f_loff_plus;
  // per subdomain face list in local (face-major) order
  std::vector<int> sub_face_off, sub_faces;
  // line ends: for subdomain i, direction d < dim, line l (other axes, lower
  // axis fastest), end e: local interface index of that end face or -1
  std::vector<int64_t> line_off;
  std::vector<int> line_g;
  int maxG = 0, maxC = 0, maxFn = 0;

  int64_t face_id(int d, int i0, int i1, int i2) const {
    return face_off[d] + i0 + (int64_t)fshape[d][0] * (i1 + (int64_t)fshape[d][1] * i2);
  }
  int64_t cell_id(int i0, int i1, int i2) const {
    return i0 + (int64_t)n[0] * (i1 + (int64_t)n[1] * i2);
  }

  void build(int dim_, const int *n_, const double *h_, const int *nsub_, const int *const *cuts_) {
    dim = dim_;
    if (dim != 2 && dim != 3) throw std::invalid_argument("dim must be 2 or 3");
    for (int d = 0; d < 3; ++d) {
      n[d] = d < dim ? n_[d] : 1;
      h[d] = d < dim ? h_[d] : 1.0;
      nsub[d] = d < dim ? nsub_[d] : 1;
      if (n[d] < 1) throw std::invalid_argument("n[d] must be >= 1");
      if (!(h[d] > 0.0)) throw std::invalid_argument("h[d] must be > 0");
      if (nsub[d] < 1 || nsub[d] > n[d]) throw std::invalid_argument("bad nsub");
      cuts[d].assign(nsub[d] + 1, 0);
      if (d < dim) {
        for (int k = 0; k <= nsub[d]; ++k) cuts[d][k] = cuts_[d][k];
      } else {
        cuts[d][1] = 1;
      }
      if (cuts[d][0] != 0 || cuts[d][nsub[d]] != n[d]) throw std::invalid_argument("cuts must span [0, n]");
      for (int k = 0; k < nsub[d]; ++k)
        if (cuts[d][k + 1] <= cuts[d][k]) throw std::invalid_argument("cuts must increase");
    }
    ncells = (int64_t)n[0] * n[1] * n[2];
    face_off[0] = 0;
    for (int d = 0; d < 3; ++d) {
      for (int e = 0; e < 3; ++e) fshape[d][e] = n[e] + (e == d ? 1 : 0);
      const int64_t cnt = d < dim ? (int64_t)fshape[d][0] * fshape[d][1] * fshape[d][2] : 0;
      face_off[d + 1] = face_off[d] + cnt;
    }
    nfaces_all = face_off[3];
    N = nsub[0] * nsub[1] * nsub[2];
    sstride[0] = 1;
    sstride[1] = nsub[0];
    sstride[2] = nsub[0] * nsub[1];

    for (int d = 0; d < 3; ++d) {
      lo[d].resize(N);
      ext[d].resize(N);
    }
    nc.resize(N);
    nG.assign(N, 0);
    nI.assign(N, 0);
    for (int i = 0; i < N; ++i) {
      int s[3] = {i % nsub[0], (i / nsub[0]) % nsub[1], i / (nsub[0] * nsub[1])};
      for (int d = 0; d < 3; ++d) {
        lo[d][i] = cuts[d][s[d]];
        ext[d][i] = cuts[d][s[d] + 1] - cuts[d][s[d]];
      }
      nc[i] = ext[0][i] * ext[1][i] * ext[2][i];
    }

    // faces: pairs (i, i + stride_d), i on the minus side; sorted by (i, j)
    std::vector<int> sub_coord(3);
    for (int i = 0; i < N; ++i) {
      int s[3] = {i % nsub[0], (i / nsub[0]) % nsub[1], i / (nsub[0] * nsub[1])};
      for (int d = 0; d < dim; ++d) {
        if (s[d] + 1 >= nsub[d]) continue;
        const int j = i + sstride[d];
        int fn = 1;
        for (int e = 0; e < 3; ++e)
          if (e != d) fn *= ext[e][i];
        f_minus.push_back(i);
        f_plus.push_back(j);
        f_n.push_back(fn);
        f_dir.push_back(d);
      }
    }
    nF = (int)f_minus.size();

    // local face order of subdomain i: -z, -y, -x, +x, +y, +z (sorted pairs)
    std::vector<std::vector<int>> minus_of(N), plus_of(N);  // faces where i is minus / plus
    for (int f = 0; f < nF; ++f) {
      minus_of[f_minus[f]].push_back(f);
      plus_of[f_plus[f]].push_back(f);
    }
    sub_face_off.assign(N + 1, 0);
    f_loff_minus.assign(nF, 0);
    f_loff_plus.assign(nF, 0);
    for (int i = 0; i < N; ++i) {
      std::vector<int> fl;
      // faces with neighbour j < i (i is the plus side), by increasing j
      std::vector<int> a = plus_of[i];
      std::sort(a.begin(), a.end(), [&](int x, int y) { return f_minus[x] < f_minus[y]; });
      std::vector<int> b = minus_of[i];
      std::sort(b.begin(), b.end(), [&](int x, int y) { return f_plus[x] < f_plus[y]; });
      fl.insert(fl.end(), a.begin(), a.end());
      fl.insert(fl.end(), b.begin(), b.end());
      int off = 0;
      for (int f : fl) {
        if (f_minus[f] == i) f_loff_minus[f] = off;
        else f_loff_plus[f] = off;
        off += f_n[f];
        sub_faces.push_back(f);
      }
      sub_face_off[i + 1] = (int)sub_faces.size();
      nG[i] = off;
    }
    g_off.assign(N + 1, 0);
    cell_off.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) {
      g_off[i + 1] = g_off[i] + nG[i];
      cell_off[i + 1] = cell_off[i] + nc[i];
    }
    lcell_global.resize(cell_off[N]);
    for (int i = 0; i < N; ++i) {
      int64_t t = cell_off[i];
      for (int z = 0; z < ext[2][i]; ++z)
        for (int y = 0; y < ext[1][i]; ++y)
          for (int x = 0; x < ext[0][i]; ++x)
            lcell_global[t++] = (int)cell_id(lo[0][i] + x, lo[1][i] + y, lo[2][i] + z);
      // interior faces: along d, ext[d]-1 per line
      int ni = 0;
      for (int d = 0; d < dim; ++d) {
        int lines = 1;
        for (int e = 0; e < 3; ++e)
          if (e != d) lines *= ext[e][i];
        ni += lines * (ext[d][i] - 1);
      }
      nI[i] = ni;
    }

    // local interface dofs: for each local face, its grid faces in grid order
    const int64_t totG = g_off[N];
    Rmap.assign(totG, -1);
    lg_dir.assign(totG, 0);
    lg_cell.assign(totG, 0);
    lg_end.assign(totG, 0);
    std::vector<int64_t> lface(totG);
    for (int i = 0; i < N; ++i) {
      for (int t = sub_face_off[i]; t < sub_face_off[i + 1]; ++t) {
        const int f = sub_faces[t];
        const int d = f_dir[f];
        const bool iminus = (f_minus[f] == i);
        const int64_t base = g_off[i] + (iminus ? f_loff_minus[f] : f_loff_plus[f]);
        // the two other axes in increasing order (grid order: lower axis fastest)
        int a0 = -1, a1 = -1;
        for (int e = 0; e < 3; ++e)
          if (e != d) { if (a0 < 0) a0 = e; else a1 = e; }
        const int pos = iminus ? lo[d][i] + ext[d][i] : lo[d][i];  // face coordinate along d
        int k = 0;
        for (int v1 = 0; v1 < ext[a1][i]; ++v1)
          for (int v0 = 0; v0 < ext[a0][i]; ++v0) {
            int c[3];
            c[d] = pos;
            c[a0] = lo[a0][i] + v0;
            c[a1] = lo[a1][i] + v1;
            const int64_t gid = face_id(d, c[0], c[1], c[2]);
            int lc[3];
            lc[d] = iminus ? ext[d][i] - 1 : 0;
            lc[a0] = v0;
            lc[a1] = v1;
            const int64_t fl = base + k;
            lface[fl] = gid;
            lg_dir[fl] = d;
            lg_cell[fl] = lc[0] + ext[0][i] * (lc[1] + ext[1][i] * lc[2]);
            lg_end[fl] = iminus ? 1 : 0;   // the face is the +d face of the minus-side cell
            ++k;
          }
      }
    }
    // interface numbering: by increasing global face id (a direct map over
    // the grid faces: mark, then number in order)
    std::vector<int> gidx(nfaces_all, -1);
    for (int64_t fl = 0; fl < totG; ++fl) gidx[lface[fl]] = 0;
    gamma_face.clear();
    for (int64_t gid = 0; gid < nfaces_all; ++gid)
      if (gidx[gid] == 0) {
        gidx[gid] = (int)gamma_face.size();
        gamma_face.push_back(gid);
      }
    nGamma = (int)gamma_face.size();
    own_minus.assign(nGamma, -1);
    own_plus.assign(nGamma, -1);
    sub_minus.assign(nGamma, -1);
    sub_plus.assign(nGamma, -1);
    for (int i = 0; i < N; ++i) {
      for (int64_t fl = g_off[i]; fl < g_off[i + 1]; ++fl) {
        const int gi = gidx[lface[fl]];
        Rmap[fl] = gi;
        if (lg_end[fl] == 1) { own_minus[gi] = (int)fl; sub_minus[gi] = i; }
        else { own_plus[gi] = (int)fl; sub_plus[gi] = i; }
      }
    }
    for (int g = 0; g < nGamma; ++g)
      if (own_minus[g] < 0 || own_plus[g] < 0) throw std::logic_error("interface dof without two owners");
    line_off.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) {
      int64_t cnt = 0;
      for (int d = 0; d < dim; ++d) cnt += 2 * (nc[i] / ext[d][i]);
      line_off[i + 1] = line_off[i] + cnt;
    }
    line_g.assign(line_off[N], -1);
    std::vector<int64_t> line_of(totG);   // first slot of the dof's line in line_g
    for (int i = 0; i < N; ++i) {
      int64_t dbase[3] = {0, 0, 0};
      int64_t acc = line_off[i];
      for (int d = 0; d < dim; ++d) {
        dbase[d] = acc;
        acc += 2 * (nc[i] / ext[d][i]);
      }
      const int st[3] = {1, ext[0][i], ext[0][i] * ext[1][i]};
      for (int t = 0; t < nG[i]; ++t) {
        const int64_t fl = g_off[i] + t;
        const int d = lg_dir[fl];
        int lc[3] = {lg_cell[fl] % ext[0][i], (lg_cell[fl] / ext[0][i]) % ext[1][i],
                     lg_cell[fl] / (ext[0][i] * ext[1][i])};
        int a0 = -1, a1 = -1;
        for (int e = 0; e < 3; ++e)
          if (e != d) { if (a0 < 0) a0 = e; else a1 = e; }
        const int l = lc[a0] + ext[a0][i] * lc[a1];
        (void)st;
        line_g[dbase[d] + 2 * l + lg_end[fl]] = t;
        line_of[fl] = dbase[d] + 2 * l;
      }
    }
    // partner: the interface dof at the opposite end of the same grid line
    lg_partner.assign(totG, -1);
    for (int64_t fl = 0; fl < totG; ++fl) lg_partner[fl] = line_g[line_of[fl] + 1 - lg_end[fl]];
    maxG = 0;
    maxC = 0;
    maxFn = 0;
    for (int i = 0; i < N; ++i) {
      maxG = std::max(maxG, nG[i]);
      maxC = std::max(maxC, nc[i]);
    }
    for (int f = 0; f < nF; ++f) maxFn = std::max(maxFn, f_n[f]);
  }
};

}  // namespace bddc
