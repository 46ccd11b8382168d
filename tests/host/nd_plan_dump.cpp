// Prints the nested-dissection plan of the coarse problem (nd.hpp) for a box
// partition with given per-face adaptive counts, for tests/test_nd_plan.py.
// usage: nd_plan_dump dim n0 n1 n2 s0 s1 s2 leaf seed [axis layer]
// With [axis layer] the faces of that subdomain plane (normal `axis`, minus
// side in subdomain layer `layer`) get 20 adaptive rows and all others none.
#include <cstdio>
#include <cstdlib>
#include <random>

#include "../../paper_1901_02090_amd/csrc/nd.hpp"

using namespace bddc;

template <class T>
static void dump(const char *name, const std::vector<T> &v) {
  printf("%s %zu", name, v.size());
  for (auto x : v) printf(" %lld", (long long)x);
  printf("\n");
}

int main(int argc, char **argv) {
  if (argc < 10) return 2;
  const int dim = atoi(argv[1]);
  int n[3], nsub[3];
  for (int d = 0; d < 3; ++d) {
    n[d] = atoi(argv[2 + d]);
    nsub[d] = atoi(argv[5 + d]);
  }
  const int leaf = atoi(argv[8]);
  std::mt19937 rng(atoi(argv[9]));
  const double h[3] = {1, 1, 1};
  std::vector<int> cuts[3];
  const int *cp[3];
  for (int d = 0; d < 3; ++d) {
    for (int k = 0; k <= nsub[d]; ++k) cuts[d].push_back((int)((long long)k * n[d] / nsub[d]));
    cp[d] = cuts[d].data();
  }
  Layout L;
  L.build(dim, n, h, nsub, cp);
  std::vector<int> fk(L.nF);
  for (auto &k : fk) k = (rng() % 8 == 0) ? (int)(rng() % 24) : (int)(rng() % 5);   // heavy-tailed
  if (argc >= 12) {
    const int ax = atoi(argv[10]), layer = atoi(argv[11]);
    for (int f = 0; f < L.nF; ++f) {
      const int s = (L.f_minus[f] / L.sstride[ax]) % L.nsub[ax];
      fk[f] = (L.f_dir[f] == ax && s == layer) ? 20 : 0;
    }
  }
  NdPlan P;
  nd_plan(L, fk, leaf, P);
  if (const char *e = getenv("ND_W1")) nd_tasks(P, P.wide4, P.wide16, atoi(e));   // single-lane rows up to $ND_W1
  if (const char *e = getenv("ND_TOP")) nd_dense_top(P, atoi(e));   // dense top block of at most $ND_TOP dofs
  if (const char *e = getenv("ND_SUB")) nd_subtrees(P, atoi(e));     // bottom subtrees of levels 0..$ND_SUB
  printf("N %d\nnF %d\nH %d\nnfr %d\nnk %d\n", L.N, L.nF, P.H, P.nfr, P.nk);
  dump("face_k", fk);
  dump("f_minus", L.f_minus);
  dump("sub_face_off", L.sub_face_off);
  dump("sub_faces", L.sub_faces);
  dump("lvl_off", P.lvl_off);
  dump("lvl_dof", P.lvl_dof);
  dump("first", P.first);
  dump("n", P.n);
  dump("m", P.m);
  dump("ch", P.ch);
  dump("b_off", P.b_off);
  dump("bidx", P.bidx);
  dump("ext", P.ext);
  dump("touch_off", P.touch_off);
  dump("touch", P.touch);
  dump("face_cofs", P.face_cofs);
  dump("pidx", P.pidx);
  dump("F_off", P.F_off);
  dump("r_off", P.r_off);
  dump("v_off", P.v_off);
  dump("gf", P.gf);
  dump("gb", P.gb);
  dump("cslot", P.cslot);
  dump("wdst", P.wdst);
  dump("xsc_off", P.xsc_off);
  dump("xsc", P.xsc);
  dump("task", P.task);
  dump("ftask_off", P.ftask_off);
  dump("btask_lo", P.btask_lo);
  dump("btask_hi", P.btask_hi);
  printf("sub_lv %d\nnsubt %d\n", P.sub_lv, P.nsubt);
  dump("stask", P.stask);
  dump("sph", P.sph);
  printf("top %d\nnt %d\n", P.top, P.nt);
  dump("tg_off", P.tg_off);
  dump("tg", P.tg);
  return 0;
}
