// Host-side setup of the library (classification, space-tree integration,
// assembly of the implicit block, dissected factor, global critical step,
// receiver weights) run on its own, so that the tests can build it with the
// address and undefined-behaviour sanitizers.  Prints the counts the tests
// compare with a library context on the same mesh.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_2310_14712_amd/csrc/internal.h"

int main(int argc, char** argv) {
  using namespace imex;
  const bool three = argc > 1 && std::strcmp(argv[1], "3d") == 0;
  HostSetup hs;
  const int dim = three ? 3 : 2;
  const int n2[3] = {7, 5, 1}, n3[3] = {5, 3, 4};
  const double extent[3] = {1.0, 1.0, 1.0};
  const int p = three ? 3 : 2;
  std::vector<double> centers, radii;
  if (three) {
    centers = {0.5, 0.45, 0.55, 0.1, 0.9, 0.1};
    radii = {0.3, 0.25};
  } else {
    centers = {0.55, 0.45, 0.2, 0.8};
    radii = {0.23, 0.12};
  }
  const double src2[3] = {0.05, 0.3, 0.0}, src3[3] = {0.1, 0.2, 0.15};
  std::string m = setup_mesh_host(hs, dim, three ? n3 : n2, extent, p, 1.0, 1.0, 1e-5, three ? 1 : 2,
                                  (int)radii.size(), centers.data(), radii.data(), three ? src3 : src2, 0.0, 0.9,
                                  0, nullptr);
  if (!m.empty()) {
    std::fprintf(stderr, "setup: %s\n", m.c_str());
    return 2;
  }
  bool notspd = false;
  m = assemble_implicit_host(hs, &notspd);
  if (!m.empty()) {
    std::fprintf(stderr, "assemble: %s\n", m.c_str());
    return 3;
  }
  const double dtg = global_critical_step(hs, 300, 1e-8);
  const double pts[6] = {0.31, 0.27, 0.4, 0.72, 0.66, 0.2};
  std::vector<int64_t> ids;
  std::vector<double> wts;
  m = sample_weights(hs, pts, 2, ids, wts);
  if (!m.empty()) {
    std::fprintf(stderr, "sample: %s\n", m.c_str());
    return 4;
  }
  // the nested-dissection factor's host solve: relative residual in S
  double relres = 0.0;
  if (hs.nd) {
    const int64_t nc = (int64_t)hs.c_nodes.size();
    std::vector<double> b(nc), x(nc);
    for (int64_t i = 0; i < nc; ++i) b[i] = 1.0 + 0.001 * (double)((i * 7919) % 1000);
    nd_solve_host(hs.ndf, b.data(), x.data());
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < nc; ++i) {
      double r = -b[i];
      for (int64_t t = hs.S.ptr[i]; t < hs.S.ptr[i + 1]; ++t) r += hs.S.val[t] * x[hs.S.col[t]];
      num += r * r;
      den += b[i] * b[i];
    }
    relres = std::sqrt(num / den);
  }
  std::printf("n_grid %lld n_d %lld n_c %lld nnz_kc %lld nnz_factor %lld components %zu weights %zu dt_global %.6e "
              "nd %d nd_relres %.3e\n",
              (long long)hs.n_grid, (long long)hs.d_nodes.size(), (long long)hs.c_nodes.size(),
              (long long)hs.Kc.val.size(), (long long)hs.nnz_factor, hs.layout.size(), wts.size(), dtg,
              hs.nd ? 1 : 0, relres);
  return 0;
}
