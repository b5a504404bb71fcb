// Host setup of the immersed Newmark IMEX discretisation (FP64, CPU).
//
//  * Cell classification and space-tree quadrature of cut cells (Section
//    "Spatial Discretization": trees refined towards the boundary, (p+1)^d
//    Gauss-Legendre points per leaf; empty cells below a fill ratio of
//    1e-10 are discarded, Section "Perforated plate").
//  * Element matrices (Eqs. Mglobal and K): uncut cells use the GLL-lumped
//    mass and the exact stiffness in Kronecker form; cut cells integrate
//    alpha rho N N and alpha rho c^2 grad N . grad N on the tree leaves.
//  * The d/c partition (Section "Partitioning of the Degrees of Freedom")
//    and the implicit block K^c, M^cc, S = M^cc + beta dt^2 K^cc (Newmark
//    IMEX flowchart), split into connected components, ordered by reverse
//    Cuthill-McKee and factorised once by envelope Cholesky.
//  * The uncut cell's critical step 2 / omega_max (Section "Critical time
//    step analysis of cut cells") from a cyclic Jacobi eigen solve.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <queue>
#include <sstream>

#include "internal.h"

#ifdef _OPENMP
#include <omp.h>
#endif

namespace imex {

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
bool Geometry::fictitious(const double* x) const {
  const size_t nb = r.size();
  for (size_t j = 0; j < nb; ++j) {
    double s = 0;
    for (int k = 0; k < dim; ++k) {
      const double d = x[k] - cx[3 * j + k];
      s += d * d;
    }
    if (s < r[j] * r[j]) return true;
  }
  return false;
}

int Geometry::box_state(const double* lo, const double* hi) const {
  bool any_cross = false;
  const size_t nb = r.size();
  for (size_t j = 0; j < nb; ++j) {
    double dmin2 = 0, dmax2 = 0;
    for (int k = 0; k < dim; ++k) {
      const double c = cx[3 * j + k];
      const double near = std::min(std::max(c, lo[k]), hi[k]);
      const double far = (std::fabs(c - lo[k]) > std::fabs(c - hi[k])) ? lo[k] : hi[k];
      dmin2 += (c - near) * (c - near);
      dmax2 += (c - far) * (c - far);
    }
    const double dmin = std::sqrt(dmin2), dmax = std::sqrt(dmax2);
    if (dmax <= r[j]) return 2;
    if (dmin < r[j] && r[j] < dmax) any_cross = true;
  }
  return any_cross ? 1 : 0;
}

bool Geometry::crossed(const double* lo, const double* hi) const {
  const size_t nb = r.size();
  for (size_t j = 0; j < nb; ++j) {
    double dmin2 = 0, dmax2 = 0;
    for (int k = 0; k < dim; ++k) {
      const double c = cx[3 * j + k];
      const double near = std::min(std::max(c, lo[k]), hi[k]);
      const double far = (std::fabs(c - lo[k]) > std::fabs(c - hi[k])) ? lo[k] : hi[k];
      dmin2 += (c - near) * (c - near);
      dmax2 += (c - far) * (c - far);
    }
    if (std::sqrt(dmin2) < r[j] && r[j] < std::sqrt(dmax2)) return true;
  }
  return false;
}

namespace {

struct Box {
  double lo[3], hi[3];
};

void tree_leaves(const Geometry& g, int dim, const Box& b, int level, int depth,
                 std::vector<Box>& out) {
  if (level < depth && g.crossed(b.lo, b.hi)) {
    double mid[3];
    for (int k = 0; k < dim; ++k) mid[k] = 0.5 * (b.lo[k] + b.hi[k]);
    for (int corner = 0; corner < (1 << dim); ++corner) {
      Box c = b;
      for (int k = 0; k < dim; ++k) {
        if (corner & (1 << k)) c.lo[k] = mid[k];
        else c.hi[k] = mid[k];
      }
      tree_leaves(g, dim, c, level + 1, depth, out);
    }
  } else {
    out.push_back(b);
  }
}

// Accumulate the consistent element matrices of one cell over the
// Gauss-Legendre points of one tree leaf.  The leaf's points form a tensor
// grid, so the sums over points are done one direction at a time; the point
// weights (quadrature weight times alpha) are not separable and enter at the
// innermost level.  Returns the physical volume (sum of weights where
// alpha = 1) for the fill ratio.
double leaf_accumulate(const HostSetup& hs, const double* clo, const Box& leaf,
                       const std::vector<double>& gx, const std::vector<double>& gw,
                       double* Me, double* Ke) {
  const int dim = hs.dim, n = hs.n, nq = n;
  // 1D tables per direction: values / physical derivatives at the points
  double B[3][kMaxN][kMaxN], D[3][kMaxN][kMaxN], Wq[3][kMaxN], Xq[3][kMaxN];
  for (int k = 0; k < dim; ++k) {
    const double half = 0.5 * (leaf.hi[k] - leaf.lo[k]);
    for (int q = 0; q < nq; ++q) {
      const double x = leaf.lo[k] + (gx[q] + 1.0) * half;
      Xq[k][q] = x;
      Wq[k][q] = gw[q] * half;
      const double xi = 2.0 * (x - clo[k]) / hs.h[k] - 1.0;
      double v[kMaxN], d[kMaxN];
      lagrange_eval(hs.ref.x, xi, v, d);
      for (int a = 0; a < n; ++a) {
        B[k][q][a] = v[a];
        D[k][q][a] = d[a] * (2.0 / hs.h[k]);
      }
    }
  }
  double phys = 0.0;
  const double rho = hs.rho, kap = hs.kappa;
  if (dim == 2) {
    const int nb = n * n;
    double Tm[kMaxN][kMaxN], Tk[kMaxN][kMaxN];
    for (int i = 0; i < nq; ++i) {
      std::memset(Tm, 0, sizeof(Tm));
      std::memset(Tk, 0, sizeof(Tk));
      for (int j = 0; j < nq; ++j) {
        const double x[3] = {Xq[0][i], Xq[1][j], 0.0};
        const bool fic = hs.geom.fictitious(x);
        const double wgt = Wq[0][i] * Wq[1][j];
        if (!fic) phys += wgt;
        const double cw = wgt * (fic ? hs.alpha_f : 1.0);
        for (int b = 0; b < n; ++b)
          for (int b2 = 0; b2 < n; ++b2) {
            Tm[b][b2] += cw * B[1][j][b] * B[1][j][b2];
            Tk[b][b2] += cw * D[1][j][b] * D[1][j][b2];
          }
      }
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          const int row = a + n * b;
          for (int b2 = 0; b2 < n; ++b2)
            for (int a2 = 0; a2 < n; ++a2) {
              const int col = a2 + n * b2;
              const double bb = B[0][i][a] * B[0][i][a2];
              const double dd = D[0][i][a] * D[0][i][a2];
              Me[row * nb + col] += rho * bb * Tm[b][b2];
              Ke[row * nb + col] += kap * (dd * Tm[b][b2] + bb * Tk[b][b2]);
            }
        }
    }
  } else {
    const int nb = n * n * n;
    const int n2 = n * n;
    // per x point: accumulators over (b, c) x (b2, c2)
    std::vector<double> YM(n2 * n2), YKy(n2 * n2), YKz(n2 * n2);
    double Zm[kMaxN][kMaxN], Zk[kMaxN][kMaxN];
    for (int i = 0; i < nq; ++i) {
      std::fill(YM.begin(), YM.end(), 0.0);
      std::fill(YKy.begin(), YKy.end(), 0.0);
      std::fill(YKz.begin(), YKz.end(), 0.0);
      for (int j = 0; j < nq; ++j) {
        std::memset(Zm, 0, sizeof(Zm));
        std::memset(Zk, 0, sizeof(Zk));
        for (int l = 0; l < nq; ++l) {
          const double x[3] = {Xq[0][i], Xq[1][j], Xq[2][l]};
          const bool fic = hs.geom.fictitious(x);
          const double wgt = Wq[0][i] * Wq[1][j] * Wq[2][l];
          if (!fic) phys += wgt;
          const double cw = wgt * (fic ? hs.alpha_f : 1.0);
          for (int c = 0; c < n; ++c)
            for (int c2 = 0; c2 < n; ++c2) {
              Zm[c][c2] += cw * B[2][l][c] * B[2][l][c2];
              Zk[c][c2] += cw * D[2][l][c] * D[2][l][c2];
            }
        }
        for (int c = 0; c < n; ++c)
          for (int b = 0; b < n; ++b) {
            const int r = b + n * c;
            for (int c2 = 0; c2 < n; ++c2)
              for (int b2 = 0; b2 < n; ++b2) {
                const int s = b2 + n * c2;
                const double bb = B[1][j][b] * B[1][j][b2];
                const double dd = D[1][j][b] * D[1][j][b2];
                YM[r * n2 + s] += bb * Zm[c][c2];
                YKy[r * n2 + s] += dd * Zm[c][c2];
                YKz[r * n2 + s] += bb * Zk[c][c2];
              }
          }
      }
      for (int r = 0; r < n2; ++r)
        for (int a = 0; a < n; ++a) {
          const int row = a + n * r;
          for (int s = 0; s < n2; ++s)
            for (int a2 = 0; a2 < n; ++a2) {
              const int col = a2 + n * s;
              const double bb = B[0][i][a] * B[0][i][a2];
              const double dd = D[0][i][a] * D[0][i][a2];
              Me[row * nb + col] += rho * bb * YM[r * n2 + s];
              Ke[row * nb + col] += kap * (dd * YM[r * n2 + s] + bb * (YKy[r * n2 + s] + YKz[r * n2 + s]));
            }
        }
    }
  }
  return phys;
}

// Largest eigenvalue of a symmetric matrix by cyclic Jacobi rotations.
double sym_max_eig(std::vector<double> A, int m) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, diag = 0;
    for (int i = 0; i < m; ++i) {
      diag += A[i * m + i] * A[i * m + i];
      for (int j = i + 1; j < m; ++j) off += A[i * m + j] * A[i * m + j];
    }
    if (off <= 1e-30 * diag) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[p * m + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[p * m + p], aqq = A[q * m + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < m; ++k) {
          const double akp = A[k * m + p], akq = A[k * m + q];
          A[k * m + p] = cs * akp - sn * akq;
          A[k * m + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < m; ++k) {
          const double apk = A[p * m + k], aqk = A[q * m + k];
          A[p * m + k] = cs * apk - sn * aqk;
          A[q * m + k] = sn * apk + cs * aqk;
        }
      }
  }
  double mx = -1e300;
  for (int i = 0; i < m; ++i) mx = std::max(mx, A[i * m + i]);
  return mx;
}

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= b;
  return r;
}

}  // namespace

// ---------------------------------------------------------------------------
// mesh setup
// ---------------------------------------------------------------------------
std::string setup_mesh_host(HostSetup& hs, int dim, const int* n_cells, const double* extent,
                            int p, double rho, double c, double alpha_f, int depth,
                            int n_holes, const double* centers, const double* radii,
                            const double* source, double dt, double cfl,
                            int n_forced, const int64_t* forced) {
  if (dim != 2 && dim != 3) return "dim must be 2 or 3";
  if (p < 1 || p > kMaxP) return "p must be in 1..7";
  if (depth < 0 || depth > 12) return "tree_depth must be in 0..12";
  if (!(rho > 0) || !(c > 0)) return "rho and c must be positive";
  if (!(alpha_f > 0) || alpha_f > 1) return "alpha_f must be in (0, 1]";
  if (n_holes < 0 || (n_holes > 0 && (!centers || !radii))) return "bad hole arrays";
  hs.dim = dim;
  hs.p = p;
  hs.n = p + 1;
  hs.rho = rho;
  hs.c = c;
  hs.kappa = rho * c * c;
  hs.alpha_f = alpha_f;
  hs.depth = depth;
  for (int k = 0; k < 3; ++k) {
    hs.ne[k] = 1;
    hs.nn[k] = 1;
    hs.h[k] = 1.0;
    hs.src[k] = 0.0;
  }
  for (int k = 0; k < dim; ++k) {
    if (n_cells[k] < 1) return "n_cells must be >= 1";
    if (!(extent[k] > 0)) return "extent must be positive";
    hs.ne[k] = n_cells[k];
    hs.nn[k] = (int64_t)n_cells[k] * p + 1;
    hs.h[k] = extent[k] / n_cells[k];
    hs.src[k] = source[k];
    if (!(source[k] >= 0 && source[k] <= extent[k])) return "source outside the box";
  }
  hs.n_cells = hs.ne[0] * hs.ne[1] * hs.ne[2];
  hs.n_grid = hs.nn[0] * hs.nn[1] * hs.nn[2];
  hs.geom.dim = dim;
  hs.geom.cx.assign(3 * (size_t)n_holes, 0.0);
  hs.geom.r.assign(n_holes, 0.0);
  for (int j = 0; j < n_holes; ++j) {
    for (int k = 0; k < dim; ++k) hs.geom.cx[3 * j + k] = centers[j * dim + k];
    if (!(radii[j] >= 0)) return "hole radius must be >= 0";
    hs.geom.r[j] = radii[j];
  }
  hs.ref = make_ref1d(p);
  const int n = hs.n;
  const int nb = (int)ipow(n, dim);

  // ---- uncut element: lumped mass and Kronecker stiffness -------------------
  hs.Ke_uncut.assign((size_t)nb * nb, 0.0);
  hs.Me_uncut_diag.assign(nb, 0.0);
  {
    const double* Kh = hs.ref.Kh.data();
    const double* Mh = hs.ref.Mh.data();
    const double* w = hs.ref.x.empty() ? nullptr : hs.ref.w.data();
    double J = 1.0;
    for (int k = 0; k < dim; ++k) J *= 0.5 * hs.h[k];
    if (dim == 2) {
      const double sx = hs.kappa * hs.h[1] / hs.h[0], sy = hs.kappa * hs.h[0] / hs.h[1];
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          const int r = a + n * b;
          hs.Me_uncut_diag[r] = rho * J * w[a] * w[b];
          for (int b2 = 0; b2 < n; ++b2)
            for (int a2 = 0; a2 < n; ++a2)
              hs.Ke_uncut[(size_t)r * nb + a2 + n * b2] =
                  sx * Kh[a * n + a2] * Mh[b * n + b2] + sy * Mh[a * n + a2] * Kh[b * n + b2];
        }
    } else {
      const double hx = hs.h[0], hy = hs.h[1], hz = hs.h[2];
      const double sx = hs.kappa * hy * hz / (2 * hx), sy = hs.kappa * hx * hz / (2 * hy),
                   sz = hs.kappa * hx * hy / (2 * hz);
      for (int cc = 0; cc < n; ++cc)
        for (int b = 0; b < n; ++b)
          for (int a = 0; a < n; ++a) {
            const int r = a + n * (b + n * cc);
            hs.Me_uncut_diag[r] = rho * J * w[a] * w[b] * w[cc];
            for (int c2 = 0; c2 < n; ++c2)
              for (int b2 = 0; b2 < n; ++b2)
                for (int a2 = 0; a2 < n; ++a2)
                  hs.Ke_uncut[(size_t)r * nb + a2 + n * (b2 + n * c2)] =
                      sx * Kh[a * n + a2] * Mh[b * n + b2] * Mh[cc * n + c2] +
                      sy * Mh[a * n + a2] * Kh[b * n + b2] * Mh[cc * n + c2] +
                      sz * Mh[a * n + a2] * Mh[b * n + b2] * Kh[cc * n + c2];
          }
    }
  }
  // critical step of an uncut cell: lambda_max(D^-1/2 K D^-1/2)
  {
    std::vector<double> A((size_t)nb * nb);
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j)
        A[(size_t)i * nb + j] = hs.Ke_uncut[(size_t)i * nb + j] /
                                std::sqrt(hs.Me_uncut_diag[i] * hs.Me_uncut_diag[j]);
    const double lam = sym_max_eig(A, nb);
    hs.dt_crit = 2.0 / std::sqrt(lam);
    if (dt > 0) hs.dt = dt;
    else {
      if (!(cfl > 0)) return "cfl must be positive when dt == 0";
      hs.dt = cfl * hs.dt_crit;
    }
  }

  // ---- classify cells; integrate cut cells ------------------------------------
  hs.cell_flag.assign(hs.n_cells, kUncut);
  hs.cut_id.assign(hs.n_cells, -1);
  std::vector<char> is_forced(hs.n_cells, 0);
  for (int i = 0; i < n_forced; ++i) {
    if (forced[i] < 0 || forced[i] >= hs.n_cells) return "forced_cut cell id out of range";
    is_forced[forced[i]] = 1;
  }
  std::vector<double> gx, gw;
  gauss_rule(n, gx, gw);
  // first pass: the state of each cell box (cheap)
  std::vector<int64_t> candidates;
  for (int64_t cid = 0; cid < hs.n_cells; ++cid) {
    const int64_t ix = cid % hs.ne[0], iy = (cid / hs.ne[0]) % hs.ne[1], iz = cid / (hs.ne[0] * hs.ne[1]);
    Box b;
    const int64_t idx[3] = {ix, iy, iz};
    for (int k = 0; k < 3; ++k) {
      b.lo[k] = idx[k] * hs.h[k];
      b.hi[k] = b.lo[k] + hs.h[k];
    }
    const int st = hs.geom.box_state(b.lo, b.hi);
    if (st == 2) hs.cell_flag[cid] = kEmpty;
    else if (st == 1 || is_forced[cid]) candidates.push_back(cid);
  }
  // second pass: tree quadrature of the candidates (parallel, deterministic)
  const int64_t ncand = (int64_t)candidates.size();
  std::vector<double> Mc((size_t)ncand * nb * nb, 0.0), Kc((size_t)ncand * nb * nb, 0.0);
  std::vector<double> eta(ncand, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t t = 0; t < ncand; ++t) {
    const int64_t cid = candidates[t];
    const int64_t ix = cid % hs.ne[0], iy = (cid / hs.ne[0]) % hs.ne[1], iz = cid / (hs.ne[0] * hs.ne[1]);
    const int64_t idx[3] = {ix, iy, iz};
    Box b;
    for (int k = 0; k < 3; ++k) {
      b.lo[k] = idx[k] * hs.h[k];
      b.hi[k] = b.lo[k] + hs.h[k];
    }
    std::vector<Box> leaves;
    tree_leaves(hs.geom, dim, b, 0, depth, leaves);
    double phys = 0.0;
    for (const Box& lf : leaves)
      phys += leaf_accumulate(hs, b.lo, lf, gx, gw, &Mc[(size_t)t * nb * nb], &Kc[(size_t)t * nb * nb]);
    double vol = 1.0;
    for (int k = 0; k < dim; ++k) vol *= hs.h[k];
    eta[t] = phys / vol;
  }
  int64_t ncut = 0;
  for (int64_t t = 0; t < ncand; ++t) {
    const int64_t cid = candidates[t];
    if (eta[t] < 1e-10) {
      hs.cell_flag[cid] = kEmpty;
      continue;
    }
    hs.cell_flag[cid] = kCut;
    hs.cut_id[cid] = ncut;
    hs.cut_cells.push_back(cid);
    ++ncut;
  }
  hs.Me_cut.assign((size_t)ncut * nb * nb, 0.0);
  hs.Ke_cut.assign((size_t)ncut * nb * nb, 0.0);
  for (int64_t t = 0; t < ncand; ++t) {
    const int64_t id = hs.cut_id[candidates[t]];
    if (id < 0) continue;
    std::memcpy(&hs.Me_cut[(size_t)id * nb * nb], &Mc[(size_t)t * nb * nb], sizeof(double) * nb * nb);
    std::memcpy(&hs.Ke_cut[(size_t)id * nb * nb], &Kc[(size_t)t * nb * nb], sizeof(double) * nb * nb);
  }
  hs.counts[0] = hs.counts[1] = hs.counts[2] = 0;
  for (int64_t cid = 0; cid < hs.n_cells; ++cid) hs.counts[hs.cell_flag[cid]]++;

  // ---- node kinds -------------------------------------------------------------
  std::vector<uint8_t> touch(hs.n_grid, 0);  // bit0: uncut cell, bit1: cut cell, bit2: empty cell
  for (int64_t cid = 0; cid < hs.n_cells; ++cid) {
    const uint8_t f = hs.cell_flag[cid];
    const uint8_t bit = (f == kCut) ? 2 : (f == kUncut ? 1 : 4);
    const int64_t ix = cid % hs.ne[0], iy = (cid / hs.ne[0]) % hs.ne[1], iz = cid / (hs.ne[0] * hs.ne[1]);
    const int nz = dim == 3 ? n : 1;
    for (int cc = 0; cc < nz; ++cc)
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          const int64_t g = (ix * p + a) + hs.nn[0] * ((iy * p + b) + hs.nn[1] * (iz * p + cc));
          touch[g] |= bit;
        }
  }
  hs.node_kind.assign(hs.n_grid, kInactive);
  hs.c_nodes.clear();
  hs.d_nodes.clear();
  hs.c_index.assign(hs.n_grid, -1);
  // d nodes whose adjacent cells are all uncut (3D: the tensor-product form
  // of the explicit kernel) and the other d nodes (next to an empty cell)
  hs.kron_mask.assign(dim == 3 ? (size_t)((hs.n_grid + 31) / 32) : 0, 0u);
  hs.kron_rest.clear();
  for (int64_t g = 0; g < hs.n_grid; ++g) {
    if (touch[g] & 2) {
      hs.node_kind[g] = kC;
      hs.c_index[g] = (int64_t)hs.c_nodes.size();
      hs.c_nodes.push_back(g);
    } else if (touch[g] & 1) {
      hs.node_kind[g] = kD;
      hs.d_nodes.push_back(g);
      if (dim == 3) {
        if (touch[g] & 4) hs.kron_rest.push_back(g);
        else hs.kron_mask[g >> 5] |= 1u << (g & 31);
      }
    }
  }
  hs.n_active = (int64_t)(hs.c_nodes.size() + hs.d_nodes.size());

  // ---- point source: f_x,i = alpha(x_s) N_i(x_s) --------------------------------
  {
    int64_t cidx[3] = {0, 0, 0};
    double xi[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
      int64_t e = (int64_t)std::floor(hs.src[k] / hs.h[k]);
      e = std::min<int64_t>(std::max<int64_t>(e, 0), hs.ne[k] - 1);
      cidx[k] = e;
      xi[k] = 2.0 * (hs.src[k] - e * hs.h[k]) / hs.h[k] - 1.0;
    }
    const int64_t cid = cidx[0] + hs.ne[0] * (cidx[1] + hs.ne[1] * cidx[2]);
    if (hs.cell_flag[cid] == kEmpty) return "the source lies in an empty cell";
    const double a_s = hs.geom.fictitious(hs.src) ? alpha_f : 1.0;
    double v[3][kMaxN];
    for (int k = 0; k < dim; ++k) lagrange_eval(hs.ref.x, xi[k], v[k], nullptr);
    hs.src_nodes.clear();
    hs.src_vals.clear();
    const int nz = dim == 3 ? n : 1;
    for (int cc = 0; cc < nz; ++cc)
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
          const int64_t g = (cidx[0] * p + a) + hs.nn[0] * ((cidx[1] * p + b) + hs.nn[1] * (cidx[2] * p + cc));
          double val = a_s * v[0][a] * v[1][b] * (dim == 3 ? v[2][cc] : 1.0);
          hs.src_nodes.push_back(g);
          hs.src_vals.push_back(val);
        }
  }
  return "";
}

// ---------------------------------------------------------------------------
// implicit block
// ---------------------------------------------------------------------------
namespace {

// cells adjacent to a grid node (non-empty only), in a fixed order
int adjacent_cells(const HostSetup& hs, int64_t g, int64_t* cells, int* local) {
  const int p = hs.p, n = hs.n;
  int64_t I[3] = {g % hs.nn[0], (g / hs.nn[0]) % hs.nn[1], g / (hs.nn[0] * hs.nn[1])};
  int64_t lo[3][2];
  int la[3][2], cnt[3];
  for (int k = 0; k < 3; ++k) {
    cnt[k] = 0;
    if (k >= hs.dim) {
      lo[k][0] = 0;
      la[k][0] = 0;
      cnt[k] = 1;
      continue;
    }
    if (I[k] % p == 0) {
      const int64_t e1 = I[k] / p - 1, e2 = I[k] / p;
      if (e1 >= 0) {
        lo[k][cnt[k]] = e1;
        la[k][cnt[k]++] = p;
      }
      if (e2 < hs.ne[k]) {
        lo[k][cnt[k]] = e2;
        la[k][cnt[k]++] = 0;
      }
    } else {
      lo[k][0] = I[k] / p;
      la[k][0] = (int)(I[k] % p);
      cnt[k] = 1;
    }
  }
  int m = 0;
  for (int cz = 0; cz < cnt[2]; ++cz)
    for (int cy = 0; cy < cnt[1]; ++cy)
      for (int cxx = 0; cxx < cnt[0]; ++cxx) {
        const int64_t cid = lo[0][cxx] + hs.ne[0] * (lo[1][cy] + hs.ne[1] * lo[2][cz]);
        if (hs.cell_flag[cid] == kEmpty) continue;
        cells[m] = cid;
        local[m] = la[0][cxx] + n * (la[1][cy] + n * la[2][cz]);
        ++m;
      }
  return m;
}

void cell_node_ids(const HostSetup& hs, int64_t cid, int64_t* ids) {
  const int p = hs.p, n = hs.n;
  const int64_t ix = cid % hs.ne[0], iy = (cid / hs.ne[0]) % hs.ne[1], iz = cid / (hs.ne[0] * hs.ne[1]);
  const int nz = hs.dim == 3 ? n : 1;
  int t = 0;
  for (int cc = 0; cc < nz; ++cc)
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < n; ++a)
        ids[t++] = (ix * p + a) + hs.nn[0] * ((iy * p + b) + hs.nn[1] * (iz * p + cc));
}

// Reverse Cuthill-McKee order of one connected component (local indices);
// *lev receives the breadth-first level (distance from the start vertex) of
// every local vertex.
std::vector<int64_t> rcm_order(const std::vector<int64_t>& verts, const Csr& A,
                               const std::vector<int64_t>& loc, std::vector<int64_t>* lev) {
  const int64_t m = (int64_t)verts.size();
  auto degree = [&](int64_t v) { return A.ptr[verts[v] + 1] - A.ptr[verts[v]]; };
  auto bfs_levels = [&](int64_t start, std::vector<int64_t>& level) {
    level.assign(m, -1);
    std::vector<int64_t> q{start};
    level[start] = 0;
    int64_t last = start;
    for (size_t h = 0; h < q.size(); ++h) {
      const int64_t v = q[h];
      last = v;
      for (int64_t k = A.ptr[verts[v]]; k < A.ptr[verts[v] + 1]; ++k) {
        const int64_t u = loc[A.col[k]];
        if (level[u] < 0) {
          level[u] = level[v] + 1;
          q.push_back(u);
        }
      }
    }
    // among the deepest level, the vertex of smallest degree
    const int64_t depth = level[last];
    int64_t best = last;
    for (int64_t v = 0; v < m; ++v)
      if (level[v] == depth && degree(v) < degree(best)) best = v;
    return std::make_pair(depth, best);
  };
  // pseudo-peripheral start (George-Liu)
  int64_t start = 0;
  for (int64_t v = 1; v < m; ++v)
    if (degree(v) < degree(start)) start = v;
  std::vector<int64_t> level;
  auto res = bfs_levels(start, level);
  for (int it = 0; it < 10; ++it) {
    auto res2 = bfs_levels(res.second, level);
    if (res2.first <= res.first) break;
    start = res.second;
    res = res2;
  }
  // Cuthill-McKee: BFS visiting neighbours by increasing degree
  std::vector<int64_t> order;
  order.reserve(m);
  std::vector<char> seen(m, 0);
  order.push_back(start);
  seen[start] = 1;
  std::vector<int64_t> nb;
  for (size_t h = 0; h < order.size(); ++h) {
    const int64_t v = order[h];
    nb.clear();
    for (int64_t k = A.ptr[verts[v]]; k < A.ptr[verts[v] + 1]; ++k) {
      const int64_t u = loc[A.col[k]];
      if (!seen[u]) {
        seen[u] = 1;
        nb.push_back(u);
      }
    }
    std::stable_sort(nb.begin(), nb.end(), [&](int64_t a, int64_t b) { return degree(a) < degree(b); });
    order.insert(order.end(), nb.begin(), nb.end());
  }
  // levels of the final breadth-first search from the chosen start
  bfs_levels(start, level);
  *lev = level;
  std::reverse(order.begin(), order.end());
  return order;
}

// Envelope (profile) Cholesky of the rows [begin, begin+size) of a CSR
// matrix with local columns.  Returns false on a non-positive pivot.
bool envelope_cholesky(const Csr& A, Component& cp) {
  const int64_t m = cp.size, b0 = cp.begin;
  cp.first.assign(m, 0);
  cp.rowoff.assign(m + 1, 0);
  for (int64_t i = 0; i < m; ++i) {
    int64_t f = i;
    for (int64_t k = A.ptr[b0 + i]; k < A.ptr[b0 + i + 1]; ++k) f = std::min(f, A.col[k] - b0);
    cp.first[i] = f;
    cp.rowoff[i + 1] = cp.rowoff[i] + (i - f + 1);
  }
  cp.L.assign(cp.rowoff[m], 0.0);
  for (int64_t i = 0; i < m; ++i) {
    double* Li = &cp.L[cp.rowoff[i]] - cp.first[i];  // Li[j] for j in [first[i], i]
    for (int64_t k = A.ptr[b0 + i]; k < A.ptr[b0 + i + 1]; ++k) {
      const int64_t j = A.col[k] - b0;
      if (j <= i) Li[j] += A.val[k];
    }
    const int64_t fi = cp.first[i];
    for (int64_t j = fi; j < i; ++j) {
      const double* Lj = &cp.L[cp.rowoff[j]] - cp.first[j];
      double s = Li[j];
      for (int64_t k = std::max(fi, cp.first[j]); k < j; ++k) s -= Li[k] * Lj[k];
      Li[j] = s / Lj[j];
    }
    double s = Li[i];
    for (int64_t k = fi; k < i; ++k) s -= Li[k] * Li[k];
    if (!(s > 0)) return false;
    Li[i] = std::sqrt(s);
  }
  return true;
}

Csr permute_sym(const Csr& A, const std::vector<int64_t>& newpos) {
  // rows and columns (both c indices) renumbered: new = newpos[old]
  const int64_t m = A.nrows;
  std::vector<int64_t> oldrow(m);
  for (int64_t i = 0; i < m; ++i) oldrow[newpos[i]] = i;
  Csr B;
  B.nrows = m;
  B.ptr.assign(m + 1, 0);
  for (int64_t i = 0; i < m; ++i) B.ptr[i + 1] = B.ptr[i] + (A.ptr[oldrow[i] + 1] - A.ptr[oldrow[i]]);
  B.col.resize(B.ptr[m]);
  B.val.resize(B.ptr[m]);
  std::vector<std::pair<int64_t, double>> tmp;
  for (int64_t i = 0; i < m; ++i) {
    tmp.clear();
    const int64_t o = oldrow[i];
    for (int64_t k = A.ptr[o]; k < A.ptr[o + 1]; ++k) tmp.emplace_back(newpos[A.col[k]], A.val[k]);
    std::sort(tmp.begin(), tmp.end());
    for (size_t t = 0; t < tmp.size(); ++t) {
      B.col[B.ptr[i] + t] = tmp[t].first;
      B.val[B.ptr[i] + t] = tmp[t].second;
    }
  }
  return B;
}

Csr permute_rows(const Csr& A, const std::vector<int64_t>& newpos) {
  const int64_t m = A.nrows;
  std::vector<int64_t> oldrow(m);
  for (int64_t i = 0; i < m; ++i) oldrow[newpos[i]] = i;
  Csr B;
  B.nrows = m;
  B.ptr.assign(m + 1, 0);
  for (int64_t i = 0; i < m; ++i) B.ptr[i + 1] = B.ptr[i] + (A.ptr[oldrow[i] + 1] - A.ptr[oldrow[i]]);
  B.col.resize(B.ptr[m]);
  B.val.resize(B.ptr[m]);
  for (int64_t i = 0; i < m; ++i) {
    const int64_t o = oldrow[i];
    std::copy(A.col.begin() + A.ptr[o], A.col.begin() + A.ptr[o + 1], B.col.begin() + B.ptr[i]);
    std::copy(A.val.begin() + A.ptr[o], A.val.begin() + A.ptr[o + 1], B.val.begin() + B.ptr[i]);
  }
  return B;
}

}  // namespace

std::string assemble_implicit_host(HostSetup& hs, bool* notspd) {
  *notspd = false;
  const int dim = hs.dim, n = hs.n;
  const int nb = (int)ipow(n, dim);
  const int64_t nc = (int64_t)hs.c_nodes.size();

  // ---- rows of K^c (grid columns) and M^cc (c columns), c order by grid id
  std::vector<std::vector<std::pair<int64_t, double>>> krow(nc), mrow(nc);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < nc; ++i) {
    const int64_t g = hs.c_nodes[i];
    int64_t cells[8];
    int local[8];
    const int m = adjacent_cells(hs, g, cells, local);
    int64_t ids[kMaxN * kMaxN * kMaxN];
    auto& kr = krow[i];
    auto& mr = mrow[i];
    for (int t = 0; t < m; ++t) {
      const int64_t cid = cells[t];
      const int li = local[t];
      cell_node_ids(hs, cid, ids);
      if (hs.cell_flag[cid] == kCut) {
        const int64_t id = hs.cut_id[cid];
        const double* Ke = &hs.Ke_cut[((size_t)id * nb + li) * nb];
        const double* Me = &hs.Me_cut[((size_t)id * nb + li) * nb];
        for (int j = 0; j < nb; ++j) {
          kr.emplace_back(ids[j], Ke[j]);
          mr.emplace_back(hs.c_index[ids[j]], Me[j]);  // all nodes of a cut cell are c nodes
        }
      } else {
        const double* Ke = &hs.Ke_uncut[(size_t)li * nb];
        for (int j = 0; j < nb; ++j) kr.emplace_back(ids[j], Ke[j]);
        mr.emplace_back(i, hs.Me_uncut_diag[li]);
      }
    }
    // reduce duplicates in a fixed order (stable sort keeps cell order)
    auto reduce = [](std::vector<std::pair<int64_t, double>>& v) {
      std::stable_sort(v.begin(), v.end(),
                       [](const std::pair<int64_t, double>& a, const std::pair<int64_t, double>& b) {
                         return a.first < b.first;
                       });
      size_t o = 0;
      for (size_t k = 0; k < v.size(); ++k) {
        if (o > 0 && v[o - 1].first == v[k].first) v[o - 1].second += v[k].second;
        else v[o++] = v[k];
      }
      v.resize(o);
    };
    reduce(kr);
    reduce(mr);
  }
  auto to_csr = [](std::vector<std::vector<std::pair<int64_t, double>>>& rows) {
    Csr A;
    A.nrows = (int64_t)rows.size();
    A.ptr.assign(A.nrows + 1, 0);
    for (int64_t i = 0; i < A.nrows; ++i) A.ptr[i + 1] = A.ptr[i] + (int64_t)rows[i].size();
    A.col.resize(A.ptr[A.nrows]);
    A.val.resize(A.ptr[A.nrows]);
    for (int64_t i = 0; i < A.nrows; ++i)
      for (size_t t = 0; t < rows[i].size(); ++t) {
        A.col[A.ptr[i] + t] = rows[i][t].first;
        A.val[A.ptr[i] + t] = rows[i][t].second;
      }
    return A;
  };
  Csr Kc0 = to_csr(krow);
  Csr Mcc0 = to_csr(mrow);
  krow.clear();
  mrow.clear();
  // K^cc (c columns) for the graph and S
  Csr Kcc0;
  Kcc0.nrows = nc;
  Kcc0.ptr.assign(nc + 1, 0);
  for (int64_t i = 0; i < nc; ++i) {
    for (int64_t k = Kc0.ptr[i]; k < Kc0.ptr[i + 1]; ++k)
      if (hs.c_index[Kc0.col[k]] >= 0) {
        Kcc0.col.push_back(hs.c_index[Kc0.col[k]]);
        Kcc0.val.push_back(Kc0.val[k]);
      }
    Kcc0.ptr[i + 1] = (int64_t)Kcc0.col.size();
  }

  // ---- connected components and RCM ----------------------------------------------
  std::vector<int64_t> comp(nc, -1);
  std::vector<std::vector<int64_t>> comp_verts;
  for (int64_t s = 0; s < nc; ++s) {
    if (comp[s] >= 0) continue;
    const int64_t id = (int64_t)comp_verts.size();
    comp_verts.emplace_back();
    auto& vs = comp_verts.back();
    std::vector<int64_t> q{s};
    comp[s] = id;
    for (size_t h = 0; h < q.size(); ++h) {
      const int64_t v = q[h];
      vs.push_back(v);
      for (int64_t k = Kcc0.ptr[v]; k < Kcc0.ptr[v + 1]; ++k) {
        const int64_t u = Kcc0.col[k];
        if (comp[u] < 0) {
          comp[u] = id;
          q.push_back(u);
        }
      }
    }
    std::sort(vs.begin(), vs.end());
  }
  const int64_t ncomp = (int64_t)comp_verts.size();
  std::vector<int64_t> newpos(nc, -1);
  std::vector<int64_t> comp_begin(ncomp + 1, 0);
  {
    std::vector<std::vector<int64_t>> orders(ncomp), levels(ncomp);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < ncomp; ++c) {
      const auto& vs = comp_verts[c];
      std::vector<int64_t> loc(nc, -1);  // only entries of this component are read
      for (size_t t = 0; t < vs.size(); ++t) loc[vs[t]] = (int64_t)t;
      orders[c] = rcm_order(vs, Kcc0, loc, &levels[c]);
    }
    // nested dissection (3D by default): geometric splits of every component
    // into supernodes in postorder (NdFactor)
    hs.nd = hs.factor_form == 2 || (hs.factor_form == 0 && dim == 3);
    std::vector<std::vector<NdTreeNode>> trees(hs.nd ? ncomp : 0);
    if (hs.nd) {
#pragma omp parallel for schedule(dynamic, 1)
      for (int64_t c = 0; c < ncomp; ++c) nd_dissect(hs, comp_verts[c], hs.nd_leaf, trees[c]);
      hs.ndf = NdFactor();
    }
    // split every component along its breadth-first levels: parts of about
    // `target` rows separated by single levels, ordered [parts..., separators...]
    hs.layout.assign(ncomp, ComponentLayout());
    int64_t pos = 0;
    for (int64_t c = 0; c < ncomp && hs.nd; ++c) {
      // nested dissection: the component's supernodes in postorder, one part
      ComponentLayout L;
      L.begin = pos;
      L.size = (int64_t)comp_verts[c].size();
      const int32_t base = (int32_t)hs.ndf.sn.size();
      for (const NdTreeNode& t : trees[c]) {
        NdSnode q{};
        q.c0 = pos;
        q.m = (int32_t)t.rows.size();
        q.parent = t.parent < 0 ? -1 : base + t.parent;
        hs.ndf.sn.push_back(q);
        for (int64_t v : t.rows) newpos[v] = pos++;
      }
      if (pos != L.begin + L.size) return "nested dissection lost rows of a component";
      L.part_begin = {0, L.size};
      L.sep_begin = L.size;
      L.sep_ptr = {L.size};
      const auto& ord = orders[c];
      L.rcm.resize(L.size);
      for (int64_t t = 0; t < L.size; ++t) L.rcm[t] = newpos[comp_verts[c][ord[t]]];
      comp_begin[c] = L.begin;
      hs.layout[c] = L;
    }
    for (int64_t c = 0; c < ncomp && !hs.nd; ++c) {
      const auto& ord = orders[c];
      const auto& lev = levels[c];
      const int64_t m = (int64_t)ord.size();
      // runs of equal level in RCM order (levels are non-increasing along it)
      std::vector<int64_t> run_begin;
      for (int64_t t = 0; t < m; ++t)
        if (t == 0 || lev[ord[t]] != lev[ord[t - 1]]) run_begin.push_back(t);
      run_begin.push_back(m);
      const int64_t nruns = (int64_t)run_begin.size() - 1;
      const int64_t avg_level = std::max<int64_t>(1, m / std::max<int64_t>(1, nruns));
      // part size: a few levels, large enough that the separators (about one
      // level each) stay a small share of the rows and below 4096 in total
      const int64_t target = std::min<int64_t>(
          std::max<int64_t>({hs.part_rows, 4 * avg_level, (m * avg_level) / 3072}), 1536);
      // role of each run: 0 = part, 1 = separator
      std::vector<int> role(nruns, 0);
      const bool split = true;
      int64_t acc = 0;
      for (int64_t r = 0; r < nruns; ++r) {
        const int64_t len = run_begin[r + 1] - run_begin[r];
        if (split && acc >= target && r + 1 < nruns) {
          role[r] = 1;
          acc = 0;
          continue;
        }
        acc += len;
      }
      // a trailing part must be large enough to be worth a separator
      for (int64_t r = nruns - 1; r >= 0; --r) {
        if (role[r] == 1) {
          int64_t tail = m - run_begin[r + 1];
          if (tail < target / 4) role[r] = 0;
          break;
        }
      }
      ComponentLayout L;
      L.begin = pos;
      L.size = m;
      std::vector<int64_t> part_nodes, sep_nodes;
      std::vector<int64_t> pb{0}, sp;
      for (int64_t r = 0; r < nruns; ++r) {
        if (role[r] == 1) {
          if (!part_nodes.empty() && pb.back() != (int64_t)part_nodes.size()) pb.push_back((int64_t)part_nodes.size());
          sp.push_back((int64_t)sep_nodes.size());
          for (int64_t t = run_begin[r]; t < run_begin[r + 1]; ++t) sep_nodes.push_back(ord[t]);
        } else {
          for (int64_t t = run_begin[r]; t < run_begin[r + 1]; ++t) part_nodes.push_back(ord[t]);
        }
      }
      if (pb.back() != (int64_t)part_nodes.size()) pb.push_back((int64_t)part_nodes.size());
      L.part_begin = pb;
      L.sep_begin = (int64_t)part_nodes.size();
      for (int64_t k : sp) L.sep_ptr.push_back(L.sep_begin + k);
      L.sep_ptr.push_back(m);
      if (sp.empty()) L.sep_ptr.assign(1, m);
      for (int64_t v : part_nodes) newpos[comp_verts[c][v]] = pos++;
      for (int64_t v : sep_nodes) newpos[comp_verts[c][v]] = pos++;
      L.rcm.resize(m);
      for (int64_t t = 0; t < m; ++t) L.rcm[t] = newpos[comp_verts[c][ord[t]]];
      comp_begin[c] = L.begin;
      hs.layout[c] = L;
    }
    comp_begin[ncomp] = pos;
  }
  // ---- apply the permutation -----------------------------------------------------
  {
    std::vector<int64_t> cn(nc);
    for (int64_t i = 0; i < nc; ++i) cn[newpos[i]] = hs.c_nodes[i];
    hs.c_nodes = cn;
    for (int64_t i = 0; i < nc; ++i) hs.c_index[hs.c_nodes[i]] = i;
  }
  hs.Kc = permute_rows(Kc0, newpos);
  Csr Kcc = permute_sym(Kcc0, newpos);
  hs.Mcc = permute_sym(Mcc0, newpos);
  hs.Kcc = Kcc;
  // K^cd: the d columns of K^c
  hs.Kcd = Csr();
  hs.Kcd.nrows = nc;
  hs.Kcd.ptr.assign(nc + 1, 0);
  for (int64_t i = 0; i < nc; ++i) {
    for (int64_t k = hs.Kc.ptr[i]; k < hs.Kc.ptr[i + 1]; ++k)
      if (hs.node_kind[hs.Kc.col[k]] == kD) {
        hs.Kcd.col.push_back(hs.Kc.col[k]);
        hs.Kcd.val.push_back(hs.Kc.val[k]);
      }
    hs.Kcd.ptr[i + 1] = (int64_t)hs.Kcd.col.size();
  }
  // S = M^cc + beta dt^2 K^cc on the pattern of K^cc (which contains that of M^cc)
  const double bdt2 = hs.beta * hs.dt * hs.dt;
  hs.S = Kcc;
  for (int64_t i = 0; i < nc; ++i) {
    for (int64_t k = hs.S.ptr[i]; k < hs.S.ptr[i + 1]; ++k) hs.S.val[k] *= bdt2;
    int64_t ks = hs.S.ptr[i];
    for (int64_t k = hs.Mcc.ptr[i]; k < hs.Mcc.ptr[i + 1]; ++k) {
      while (ks < hs.S.ptr[i + 1] && hs.S.col[ks] < hs.Mcc.col[k]) ++ks;
      if (ks == hs.S.ptr[i + 1] || hs.S.col[ks] != hs.Mcc.col[k]) return "M^cc pattern not contained in K^cc";
      hs.S.val[ks] += hs.Mcc.val[k];
    }
  }
  // f_x on c dofs
  hs.fxc.assign(nc, 0.0);
  for (size_t t = 0; t < hs.src_nodes.size(); ++t) {
    const int64_t ci = hs.c_index[hs.src_nodes[t]];
    if (ci >= 0) hs.fxc[ci] = hs.src_vals[t];
  }
  // ---- factorise M^cc (host, initial state) and S (dissected, device) ---------------
  // M^cc is factorised per component in reverse Cuthill-McKee order (banded
  // envelope); the dissected order would give separator rows spanning the
  // whole component
  hs.comps_m.assign(ncomp, Component());
  std::vector<char> ok(ncomp, 1);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < ncomp; ++c) {
    const ComponentLayout& L = hs.layout[c];
    const int64_t m = L.size;
    std::vector<int64_t> pos_in_rcm(m);
    for (int64_t t = 0; t < m; ++t) pos_in_rcm[L.rcm[t] - L.begin] = t;
    Csr B;
    B.nrows = m;
    B.ptr.assign(m + 1, 0);
    std::vector<std::pair<int64_t, double>> row;
    for (int64_t t = 0; t < m; ++t) {
      const int64_t i = L.rcm[t];
      row.clear();
      for (int64_t k = hs.Mcc.ptr[i]; k < hs.Mcc.ptr[i + 1]; ++k)
        row.emplace_back(pos_in_rcm[hs.Mcc.col[k] - L.begin], hs.Mcc.val[k]);
      std::sort(row.begin(), row.end());
      for (auto& e : row) {
        B.col.push_back(e.first);
        B.val.push_back(e.second);
      }
      B.ptr[t + 1] = (int64_t)B.col.size();
    }
    hs.comps_m[c].begin = 0;
    hs.comps_m[c].size = m;
    if (!envelope_cholesky(B, hs.comps_m[c])) ok[c] = 0;
    hs.comps_m[c].begin = L.begin;
  }
  for (int64_t c = 0; c < ncomp; ++c)
    if (!ok[c]) {
      *notspd = true;
      std::ostringstream os;
      os << "Cholesky factorisation of M^cc failed (non-positive pivot) in component " << c;
      return os.str();
    }
  if (hs.nd) {
    int threads = 1;
#ifdef _OPENMP
    threads = omp_get_max_threads();
#endif
    std::string m = build_nd_factor(hs.S, hs.ndf, threads);
    if (!m.empty()) {
      *notspd = m.find("non-positive pivot") != std::string::npos;
      return m;
    }
    hs.fac = DissectedFactor();
    hs.nnz_factor = hs.ndf.nnz_L;
    return "";
  }
  std::string m = build_dissected_factor(hs.S, hs.layout, hs.fac, hs.dense_rows, hs.dense_inverse,
                                         hs.device_inverse_min, hs.inverse_device);
  if (!m.empty()) {
    *notspd = true;
    return m;
  }
  hs.nnz_factor = hs.fac.nnz_total;
  return "";
}

void envelope_solve(const std::vector<Component>& comps, double* x) {
  for (const Component& cp : comps) {
    double* v = x + cp.begin;
    const int64_t m = cp.size;
    for (int64_t i = 0; i < m; ++i) {  // L y = b
      const double* Li = &cp.L[cp.rowoff[i]] - cp.first[i];
      double s = v[i];
      for (int64_t k = cp.first[i]; k < i; ++k) s -= Li[k] * v[k];
      v[i] = s / Li[i];
    }
    for (int64_t i = m - 1; i >= 0; --i) {  // L^T x = y (column sweep)
      const double* Li = &cp.L[cp.rowoff[i]] - cp.first[i];
      v[i] /= Li[i];
      for (int64_t k = cp.first[i]; k < i; ++k) v[k] -= Li[k] * v[i];
    }
  }
}

void mcc_solve(const HostSetup& hs, double* x) {
  for (size_t c = 0; c < hs.layout.size(); ++c) {
    const ComponentLayout& L = hs.layout[c];
    std::vector<double> v(L.size);
    for (int64_t t = 0; t < L.size; ++t) v[t] = x[L.rcm[t]];
    Component cp = hs.comps_m[c];
    cp.begin = 0;
    std::vector<Component> one{cp};
    envelope_solve(one, v.data());
    for (int64_t t = 0; t < L.size; ++t) x[L.rcm[t]] = v[t];
  }
}

std::string sample_weights(const HostSetup& hs, const double* pts, int64_t n, std::vector<int64_t>& ids,
                           std::vector<double>& wts) {
  const int nb = (int)ipow(hs.n, hs.dim);
  ids.assign((size_t)n * nb, 0);
  wts.assign((size_t)n * nb, 0.0);
  std::vector<double> val(3 * kMaxN), der(kMaxN);
  for (int64_t r = 0; r < n; ++r) {
    int64_t cidx[3] = {0, 0, 0};
    for (int k = 0; k < hs.dim; ++k) {
      const double x = pts[r * hs.dim + k];
      if (!(x >= 0.0 && x <= hs.ne[k] * hs.h[k])) return "a sample point lies outside the box";
      cidx[k] = std::min<int64_t>((int64_t)std::floor(x / hs.h[k]), hs.ne[k] - 1);
      const double xi = 2.0 * (x - cidx[k] * hs.h[k]) / hs.h[k] - 1.0;
      lagrange_eval(hs.ref.x, xi, &val[k * kMaxN], der.data());
    }
    const int64_t cid = cidx[0] + hs.ne[0] * (cidx[1] + hs.ne[1] * cidx[2]);
    if (hs.cell_flag[cid] == kEmpty) return "a sample point lies in an empty cell";
    cell_node_ids(hs, cid, &ids[(size_t)r * nb]);
    for (int t = 0; t < nb; ++t) {  // local node t = a + n b (+ n^2 c)
      double v = val[t % hs.n] * val[kMaxN + (t / hs.n) % hs.n];
      if (hs.dim == 3) v *= val[2 * kMaxN + t / (hs.n * hs.n)];
      wts[(size_t)r * nb + t] = v;
    }
  }
  return "";
}

double global_critical_step(const HostSetup& hs, int max_iter, double rel_tol) {
  const int nb = (int)ipow(hs.n, hs.dim);
  const int64_t ng = hs.n_grid;
  // lumped mass of the d nodes (their cells are all uncut)
  std::vector<double> md(ng, 0.0);
  for (int64_t g : hs.d_nodes) {
    int64_t cells[8];
    int local[8];
    const int m = adjacent_cells(hs, g, cells, local);
    for (int t = 0; t < m; ++t) md[g] += hs.Me_uncut_diag[local[t]];
  }
  auto k_apply = [&](const std::vector<double>& u, std::vector<double>& y) {
    std::fill(y.begin(), y.end(), 0.0);
    int64_t ids[kMaxN * kMaxN * kMaxN];
    std::vector<double> ue(nb);
    for (int64_t cid = 0; cid < (int64_t)hs.cell_flag.size(); ++cid) {
      if (hs.cell_flag[cid] == kEmpty) continue;
      cell_node_ids(hs, cid, ids);
      for (int j = 0; j < nb; ++j) ue[j] = u[ids[j]];
      const double* Ke = hs.cell_flag[cid] == kCut ? &hs.Ke_cut[(size_t)hs.cut_id[cid] * nb * nb] : hs.Ke_uncut.data();
      for (int i = 0; i < nb; ++i) {
        double s = 0.0;
        for (int j = 0; j < nb; ++j) s += Ke[(size_t)i * nb + j] * ue[j];
        y[ids[i]] += s;
      }
    }
  };
  auto m_apply = [&](const std::vector<double>& u, std::vector<double>& y) {  // block mass
    std::fill(y.begin(), y.end(), 0.0);
    for (int64_t g : hs.d_nodes) y[g] = md[g] * u[g];
    for (int64_t i = 0; i < hs.Mcc.nrows; ++i) {
      double s = 0.0;
      for (int64_t k = hs.Mcc.ptr[i]; k < hs.Mcc.ptr[i + 1]; ++k) s += hs.Mcc.val[k] * u[hs.c_nodes[hs.Mcc.col[k]]];
      y[hs.c_nodes[i]] = s;
    }
  };
  auto m_solve = [&](std::vector<double>& y) {  // y <- M^-1 y on the active dofs
    for (int64_t g : hs.d_nodes) y[g] /= md[g];
    std::vector<double> yc(hs.c_nodes.size());
    for (size_t i = 0; i < yc.size(); ++i) yc[i] = y[hs.c_nodes[i]];
    mcc_solve(hs, yc.data());
    for (size_t i = 0; i < yc.size(); ++i) y[hs.c_nodes[i]] = yc[i];
  };
  // seeded start on the active dofs (splitmix64 to uniform in [-1, 1))
  std::vector<double> x(ng, 0.0), y(ng), mx(ng);
  uint64_t st = 0x9E3779B97F4A7C15ULL;
  auto next = [&]() {
    uint64_t z = (st += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  };
  for (int64_t g : hs.d_nodes) x[g] = next();
  for (int64_t g : hs.c_nodes) x[g] = next();
  double lam = 0.0;
  for (int it = 0; it < max_iter; ++it) {
    // Rayleigh quotient x^T K x / x^T M x, then x <- M^-1 K x, M-normalised
    k_apply(x, y);
    m_apply(x, mx);
    double xkx = 0.0, xmx = 0.0;
    for (int64_t g = 0; g < ng; ++g) {
      xkx += x[g] * y[g];
      xmx += x[g] * mx[g];
    }
    const double lam_new = xkx / xmx;
    const bool done = it > 0 && std::fabs(lam_new - lam) <= rel_tol * lam_new;
    lam = lam_new;
    if (done) break;
    m_solve(y);
    m_apply(y, mx);
    double nrm = 0.0;
    for (int64_t g = 0; g < ng; ++g) nrm += y[g] * mx[g];
    nrm = std::sqrt(nrm);
    for (int64_t g = 0; g < ng; ++g) x[g] = y[g] / nrm;
  }
  return 2.0 / std::sqrt(lam);
}

void kc_apply(const HostSetup& hs, const double* u, double* y) {
  for (int64_t i = 0; i < hs.Kc.nrows; ++i) {
    double s = 0;
    for (int64_t k = hs.Kc.ptr[i]; k < hs.Kc.ptr[i + 1]; ++k) s += hs.Kc.val[k] * u[hs.Kc.col[k]];
    y[i] = s;
  }
}

// ---------------------------------------------------------------------------
// dissected factor for the device
// ---------------------------------------------------------------------------
namespace {

// principal submatrix of A on the rows / columns [b, e), local indices
Csr principal(const Csr& A, int64_t b, int64_t e) {
  Csr B;
  B.nrows = e - b;
  B.ptr.assign(B.nrows + 1, 0);
  for (int64_t i = b; i < e; ++i) {
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (A.col[k] >= b && A.col[k] < e) {
        B.col.push_back(A.col[k] - b);
        B.val.push_back(A.val[k]);
      }
    B.ptr[i - b + 1] = (int64_t)B.col.size();
  }
  return B;
}

// Envelope Cholesky of a local matrix and its device chain: the envelope
// values, the inverses of the kBlk x kBlk diagonal blocks (lower triangles
// packed by columns), and per-row / per-block metadata.
bool make_chain(const Csr& A, int64_t row0, int comp, Component& cp, DissectedFactor& F, ChainMeta& cm) {
  const int64_t m = A.nrows;
  cp.begin = 0;
  cp.size = m;
  cm = ChainMeta{};
  cm.row0 = row0;
  cm.nrows = (int32_t)m;
  cm.comp = comp;
  cm.zoff = -1;
  if (m == 0) return true;
  if (!envelope_cholesky(A, cp)) return false;
  const int nb = (int)((m + kBlk - 1) / kBlk);
  cm.nblocks = nb;
  cm.nnz = (int32_t)cp.L.size();
  cm.voff = (int64_t)F.vals.size();
  cm.ioff = (int64_t)F.ints.size();
  F.vals.insert(F.vals.end(), cp.L.begin(), cp.L.end());
  auto Lij = [&](int64_t i, int64_t j) -> double {
    if (j < cp.first[i] || j > i) return 0.0;
    return cp.L[cp.rowoff[i] + (j - cp.first[i])];
  };
  std::vector<double> Dall((size_t)nb * kBlk * kBlk);
  for (int b = 0; b < nb; ++b) {
    const int64_t r0 = (int64_t)b * kBlk;
    const int nr = (int)std::min<int64_t>(kBlk, m - r0);
    double* Dm = &Dall[(size_t)b * kBlk * kBlk];  // Dm[r * kBlk + c] = D(r, c)
    for (int cidx = 0; cidx < kBlk; ++cidx) {
      for (int r = 0; r < kBlk; ++r) Dm[r * kBlk + cidx] = 0.0;
      if (cidx >= nr) {
        Dm[cidx * kBlk + cidx] = 1.0;
        continue;
      }
      for (int r = cidx; r < nr; ++r) {  // forward substitution L_bb x = e_c
        double sacc = (r == cidx) ? 1.0 : 0.0;
        for (int k = cidx; k < r; ++k) sacc -= Lij(r0 + r, r0 + k) * Dm[k * kBlk + cidx];
        Dm[r * kBlk + cidx] = sacc / Lij(r0 + r, r0 + r);
      }
    }
    for (int cidx = 0; cidx < kBlk; ++cidx)  // packed by columns: (r, c), r >= c
      for (int r = cidx; r < kBlk; ++r) F.vals.push_back(Dm[r * kBlk + cidx]);
  }
  for (int64_t i = 0; i < m; ++i) F.ints.push_back((int32_t)cp.first[i]);
  for (int64_t i = 0; i < m; ++i) F.ints.push_back((int32_t)cp.rowoff[i]);
  for (int b = 0; b < nb; ++b) {
    const int64_t rend = std::min<int64_t>((int64_t)(b + 1) * kBlk, m);
    int64_t rmax = rend - 1;
    for (int64_t j = rend; j < m; ++j)
      if (cp.first[j] < rend) rmax = j;
    F.ints.push_back((int32_t)rmax);
  }
  const int64_t nv = cm.nnz + (int64_t)nb * kTri, ni = 2 * m + nb;
  F.max_chain_doubles = std::max(F.max_chain_doubles, nv);
  F.max_chain_ints = std::max(F.max_chain_ints, ni);
  F.max_chain_rows = std::max<int64_t>(F.max_chain_rows, m);
  return true;
}

}  // namespace

namespace {

// dense Cholesky (lower, row-major) and inverse of an SPD matrix; false on a
// non-positive pivot
bool dense_spd_inverse(std::vector<double>& A, int64_t n, std::vector<double>& inv) {
  for (int64_t j = 0; j < n; ++j) {
    double* Lj = &A[j * n];
    double d = Lj[j];
    for (int64_t k = 0; k < j; ++k) d -= Lj[k] * Lj[k];
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    Lj[j] = d;
    for (int64_t i = j + 1; i < n; ++i) {
      double* Li = &A[i * n];
      double sacc = Li[j];
      for (int64_t k = 0; k < j; ++k) sacc -= Li[k] * Lj[k];
      Li[j] = sacc / d;
    }
  }
  // L^-1 by rows (forward substitution), then inv = L^-T L^-1
  std::vector<double> Li((size_t)n * n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    Li[i * n + i] = 1.0 / A[i * n + i];
    for (int64_t j = 0; j < i; ++j) {
      double sacc = 0.0;
      for (int64_t k = j; k < i; ++k) sacc += A[i * n + k] * Li[k * n + j];
      Li[i * n + j] = -sacc / A[i * n + i];
    }
  }
  inv.assign((size_t)n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      double sacc = 0.0;
      for (int64_t k = i; k < n; ++k) sacc += Li[k * n + i] * Li[k * n + j];
      inv[i * n + j] = sacc;
      inv[j * n + i] = sacc;
    }
  return true;
}

// everything one component contributes to the dissected factor, with local
// offsets; merged in component order afterwards
struct CompPiece {
  DissectedFactor F;
  std::vector<std::pair<int64_t, int64_t>> sep_src;  // (global c row, local slot)
  std::string err;
};

void build_component(const Csr& S, const ComponentLayout& L, int ci, bool dense, int64_t dense_rows,
                     DenseInverseFn inverse, int64_t inverse_min, int inverse_device, CompPiece& out) {
  DissectedFactor& F = out.F;
  const int64_t b = L.begin;
  const int64_t nparts = (int64_t)L.part_begin.size() - 1;
  const int64_t nsep = L.size - L.sep_begin;
  std::vector<double> Sig((size_t)nsep * nsep, 0.0);
  for (int64_t s = 0; s < nsep; ++s) {
    const int64_t i = b + L.sep_begin + s;
    for (int64_t k = S.ptr[i]; k < S.ptr[i + 1]; ++k) {
      const int64_t j = S.col[k] - b;
      if (j >= L.sep_begin && j < L.size) Sig[s * nsep + (j - L.sep_begin)] += S.val[k];
    }
  }
  int64_t coup_slots = 0;
  for (int64_t p = 0; p < nparts; ++p) {
    const int64_t pb = L.part_begin[p], pe = L.part_begin[p + 1];
    const int64_t np = pe - pb;
    Csr A = principal(S, b + pb, b + pe);
    Component cp;
    ChainMeta cm;
    if (!make_chain(A, b + pb, ci, cp, F, cm)) {
      std::ostringstream os;
      os << "Cholesky factorisation failed (non-positive pivot) in component " << ci << ", part " << p;
      out.err = os.str();
      return;
    }
    std::vector<Component> one{cp};
    cm.doff = -1;
    if (dense) {
      cm.doff = (int64_t)F.pinv.size();
      F.pinv.resize(F.pinv.size() + (size_t)np * np);
      double* P = &F.pinv[cm.doff];
      if (inverse && np > inverse_min) {
        // large part: its dense block inverted on the device
        std::fill(P, P + (size_t)np * np, 0.0);
        for (int64_t i = 0; i < np; ++i)
          for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) P[i * np + A.col[k]] = A.val[k];
        if (!inverse(P, np, inverse_device)) {
          std::ostringstream os;
          os << "dense inverse failed (non-positive pivot) in component " << ci << ", part " << p;
          out.err = os.str();
          return;
        }
      } else {
        // A_pp^-1 from the envelope factor, column by column (symmetric)
        std::vector<double> e(np);
        for (int64_t t = 0; t < np; ++t) {
          std::fill(e.begin(), e.end(), 0.0);
          e[t] = 1.0;
          envelope_solve(one, e.data());
          for (int64_t i = 0; i < np; ++i) P[i * np + t] = e[i];
        }
      }
    }
    if (nsep > 0) {
      // adjacent separators: k = p - 1 and k = p (when they exist)
      const int64_t k0 = std::max<int64_t>(p - 1, 0);
      const int64_t k1 = std::min<int64_t>(p, (int64_t)L.sep_ptr.size() - 2);
      const int64_t a0 = L.sep_ptr[k0], a1 = L.sep_ptr[k1 + 1];
      cm.adj0 = b + a0;
      cm.nadj = (int32_t)(a1 - a0);
      cm.zoff = (int64_t)F.zvals.size();
      std::vector<double> Z((size_t)np * cm.nadj, 0.0);
      for (int64_t t = 0; t < cm.nadj; ++t) {  // Z_p[:, t] = A_pp^-1 A_p,s
        const int64_t srow = b + a0 + t;
        double* z = &Z[(size_t)t * np];
        for (int64_t k = S.ptr[srow]; k < S.ptr[srow + 1]; ++k) {
          const int64_t j = S.col[k] - b;
          if (j >= pb && j < pe) z[j - pb] = S.val[k];
        }
        envelope_solve(one, z);
      }
      // Sigma[s, t] -= sum_i S[s, i] Z_p[i, t]
      for (int64_t sidx = 0; sidx < cm.nadj; ++sidx) {
        const int64_t srow = b + a0 + sidx;
        double* Srow = &Sig[(a0 - L.sep_begin + sidx) * nsep + (a0 - L.sep_begin)];
        for (int64_t k = S.ptr[srow]; k < S.ptr[srow + 1]; ++k) {
          const int64_t j = S.col[k] - b;
          if (j < pb || j >= pe) continue;
          const double v = S.val[k];
          const double* Zj = &Z[j - pb];
          for (int64_t t = 0; t < cm.nadj; ++t) Srow[t] -= v * Zj[(size_t)t * np];
        }
      }
      F.zvals.insert(F.zvals.end(), Z.begin(), Z.end());
      // A_Sp (local columns) and the contribution slots of its rows
      cm.coff = coup_slots;
      F.cp_rowptr.push_back((int64_t)F.cp_ptr.size());
      F.cp_ptr.push_back((int32_t)F.cp_col.size());
      for (int64_t t = 0; t < cm.nadj; ++t) {
        const int64_t srow = b + a0 + t;
        for (int64_t k = S.ptr[srow]; k < S.ptr[srow + 1]; ++k) {
          const int64_t j = S.col[k] - b;
          if (j >= pb && j < pe) {
            F.cp_col.push_back((int32_t)(j - pb));
            F.cp_val.push_back(S.val[k]);
          }
        }
        F.cp_ptr.push_back((int32_t)F.cp_col.size());
        out.sep_src.emplace_back(srow, coup_slots + t);
      }
      coup_slots += cm.nadj;
    } else {
      cm.adj0 = 0;
      cm.nadj = 0;
      cm.coff = -1;
      F.cp_rowptr.push_back((int64_t)F.cp_ptr.size());
      F.cp_ptr.push_back((int32_t)F.cp_col.size());
    }
    F.parts.push_back(cm);
  }
  F.coupling_slots = coup_slots;
  // inverse of the separator system from its Cholesky factor
  ChainMeta cm{};
  cm.row0 = b + L.sep_begin;
  cm.nrows = (int32_t)nsep;
  cm.comp = ci;
  cm.zoff = -1;
  cm.doff = -1;
  cm.voff = 0;
  if (nsep > dense_rows) {
    // large separator system: envelope Cholesky of Sigma (block tridiagonal
    // over the separators, so its envelope is banded) as a chain
    Csr A;
    A.nrows = nsep;
    A.ptr.assign(nsep + 1, 0);
    for (int64_t r = 0; r < nsep; ++r) {
      for (int64_t t = 0; t < nsep; ++t)
        if (Sig[r * nsep + t] != 0.0) {
          A.col.push_back(t);
          A.val.push_back(Sig[r * nsep + t]);
        }
      A.ptr[r + 1] = (int64_t)A.col.size();
    }
    Component cps;
    ChainMeta cc;
    if (!make_chain(A, b + L.sep_begin, ci, cps, F, cc)) {
      std::ostringstream os;
      os << "Cholesky factorisation of the separator system failed in component " << ci;
      out.err = os.str();
      return;
    }
    cc.zoff = -1;
    cc.doff = -1;
    cc.coff = -2;  // marks a chain-form separator system
    F.schur.push_back(cc);
    return;
  }
  bool inv_ok = true;
  if (nsep > 0 && inverse && nsep > inverse_min) {
    inv_ok = inverse(Sig.data(), nsep, inverse_device);  // large separator system: on the device
    if (inv_ok) F.schur_inv.swap(Sig);
  } else if (nsep > 0) {
    inv_ok = dense_spd_inverse(Sig, nsep, F.schur_inv);
  }
  if (!inv_ok) {
    std::ostringstream os;
    os << "Cholesky factorisation of the separator system failed in component " << ci;
    out.err = os.str();
    return;
  }
  cm.coff = -1;
  F.schur.push_back(cm);
}

}  // namespace

std::string build_dissected_factor(const Csr& S, const std::vector<ComponentLayout>& comps,
                                   DissectedFactor& F, int64_t dense_rows, DenseInverseFn inverse,
                                   int64_t inverse_min, int inverse_device) {
  F = DissectedFactor();
  const int64_t nc = S.nrows;
  F.dense = true;
  for (const ComponentLayout& L : comps)
    for (size_t p = 0; p + 1 < L.part_begin.size(); ++p)
      if (L.part_begin[p + 1] - L.part_begin[p] > dense_rows) F.dense = false;
  const int64_t ncomp = (int64_t)comps.size();
  std::vector<CompPiece> pieces(ncomp);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t ci = 0; ci < ncomp; ++ci)
    build_component(S, comps[ci], (int)ci, F.dense, dense_rows, inverse, inverse_min, inverse_device, pieces[ci]);
  for (int64_t ci = 0; ci < ncomp; ++ci)
    if (!pieces[ci].err.empty()) return pieces[ci].err;
  if (const char* dbg = std::getenv("IMEX_DEBUG"); dbg && dbg[0] == '1')
    for (int64_t ci = 0; ci < ncomp; ++ci) {
      const ComponentLayout& L = comps[ci];
      int64_t pmax = 0;
      for (size_t p = 0; p + 1 < L.part_begin.size(); ++p)
        pmax = std::max<int64_t>(pmax, L.part_begin[p + 1] - L.part_begin[p]);
      std::fprintf(stderr, "[imex] component %lld: %lld rows, %zu parts (largest %lld), %lld separator rows\n",
                   (long long)ci, (long long)L.size, L.part_begin.size() - 1, (long long)pmax,
                   (long long)(L.size - L.sep_begin));
    }
  // merge in component order, shifting the local offsets
  F.sep_src.assign(2 * nc, -1);
  int64_t slot0 = 0;
  for (int64_t ci = 0; ci < ncomp; ++ci) {
    DissectedFactor& P = pieces[ci].F;
    const int64_t voff = (int64_t)F.vals.size(), ioff = (int64_t)F.ints.size();
    const int64_t zoff = (int64_t)F.zvals.size(), doff = (int64_t)F.pinv.size();
    const int64_t soff = (int64_t)F.schur_inv.size(), cpoff = (int64_t)F.cp_ptr.size();
    const int64_t cpcol = (int64_t)F.cp_col.size();
    for (ChainMeta cm : P.parts) {
      if (cm.nrows > 0) {
        cm.voff += voff;
        cm.ioff += ioff;
      }
      if (cm.zoff >= 0) cm.zoff += zoff;
      if (cm.doff >= 0) cm.doff += doff;
      if (cm.coff >= 0) cm.coff += slot0;
      F.parts.push_back(cm);
    }
    for (ChainMeta cm : P.schur) {
      if (cm.coff == -2) {  // chain form
        cm.voff += voff;
        cm.ioff += ioff;
      } else {
        cm.voff = soff;
      }
      F.schur.push_back(cm);
    }
    F.vals.insert(F.vals.end(), P.vals.begin(), P.vals.end());
    F.ints.insert(F.ints.end(), P.ints.begin(), P.ints.end());
    F.zvals.insert(F.zvals.end(), P.zvals.begin(), P.zvals.end());
    F.pinv.insert(F.pinv.end(), P.pinv.begin(), P.pinv.end());
    F.schur_inv.insert(F.schur_inv.end(), P.schur_inv.begin(), P.schur_inv.end());
    for (int64_t v : P.cp_rowptr) F.cp_rowptr.push_back(v + cpoff);
    for (int32_t v : P.cp_ptr) F.cp_ptr.push_back((int32_t)(v + cpcol));
    F.cp_col.insert(F.cp_col.end(), P.cp_col.begin(), P.cp_col.end());
    F.cp_val.insert(F.cp_val.end(), P.cp_val.begin(), P.cp_val.end());
    for (const auto& e : pieces[ci].sep_src) {
      int64_t* src = &F.sep_src[2 * e.first];
      if (src[0] < 0) src[0] = slot0 + e.second;
      else src[1] = slot0 + e.second;
    }
    slot0 += P.coupling_slots;
    F.max_chain_doubles = std::max(F.max_chain_doubles, P.max_chain_doubles);
    F.max_chain_ints = std::max(F.max_chain_ints, P.max_chain_ints);
    F.max_chain_rows = std::max(F.max_chain_rows, P.max_chain_rows);
    DissectedFactor().parts.swap(P.parts);  // release memory early
    std::vector<double>().swap(P.vals);
    std::vector<double>().swap(P.pinv);
    std::vector<double>().swap(P.zvals);
    std::vector<double>().swap(P.schur_inv);
  }
  F.coupling_slots = slot0;
  for (size_t ci = 0; ci < F.schur.size(); ++ci) {
    const int64_t nsep = F.schur[ci].nrows;
    if (F.schur[ci].coff == -2) {
      F.schur_chain.push_back((int64_t)ci);
      continue;
    }
    for (int64_t r0 = 0; r0 < nsep; r0 += 16) {
      F.schur_chunks.push_back((int64_t)ci);
      F.schur_chunks.push_back(r0);
    }
  }
  for (size_t p = 0; p < F.parts.size(); ++p)
    for (int64_t r0 = 0; r0 < F.parts[p].nrows; r0 += 64) {
      F.part_chunks.push_back((int64_t)p);
      F.part_chunks.push_back(r0);
    }
  if (F.dense)
    for (size_t p = 0; p < F.parts.size(); ++p) {
      for (int64_t r0 = 0; r0 < F.parts[p].nrows; r0 += 16) {
        F.dense_chunks.push_back(0);
        F.dense_chunks.push_back((int64_t)p);
        F.dense_chunks.push_back(r0);
      }
      for (int64_t k0 = 0; k0 < F.parts[p].nadj; k0 += 16) {
        F.dense_chunks.push_back(1);
        F.dense_chunks.push_back((int64_t)p);
        F.dense_chunks.push_back(k0);
      }
    }
  F.nnz_total = (int64_t)((F.dense ? F.pinv.size() : F.vals.size()) + F.zvals.size() + F.schur_inv.size());
  return "";
}

std::string build_lts_rows(const HostSetup& hs, LtsRows& out) {
  const int64_t nc = (int64_t)hs.c_nodes.size();
  const int nb = (int)ipow(hs.n, hs.dim);
  out = LtsRows();
  out.nc = nc;
  // d neighbours of the c dofs: the d columns of K^c
  std::vector<int64_t> nd(hs.Kcd.col.begin(), hs.Kcd.col.end());
  std::sort(nd.begin(), nd.end());
  nd.erase(std::unique(nd.begin(), nd.end()), nd.end());
  out.node = hs.c_nodes;
  out.node.insert(out.node.end(), nd.begin(), nd.end());
  const int64_t nf = (int64_t)out.node.size();
  out.Ko.nrows = out.Kf.nrows = nf;
  out.Ko.ptr.assign(nf + 1, 0);
  out.Kf.ptr.assign(nf + 1, 0);
  out.mass.assign(nf, 0.0);
  std::vector<std::pair<int64_t, double>> row;
  auto push = [&](int64_t r) {
    for (const auto& e : row) {
      const int64_t ci = hs.c_index[e.first];
      if (ci >= 0) {
        out.Kf.col.push_back(ci);
        out.Kf.val.push_back(e.second);
      } else {
        out.Ko.col.push_back(e.first);
        out.Ko.val.push_back(e.second);
      }
    }
    out.Ko.ptr[r + 1] = (int64_t)out.Ko.col.size();
    out.Kf.ptr[r + 1] = (int64_t)out.Kf.col.size();
  };
  for (int64_t i = 0; i < nc; ++i) {
    row.clear();
    for (int64_t k = hs.Kc.ptr[i]; k < hs.Kc.ptr[i + 1]; ++k) row.emplace_back(hs.Kc.col[k], hs.Kc.val[k]);
    push(i);
    for (int64_t k = hs.Mcc.ptr[i]; k < hs.Mcc.ptr[i + 1]; ++k) {
      if (hs.Mcc.col[k] == i) out.mass[i] = hs.Mcc.val[k];
      else if (hs.Mcc.val[k] != 0.0) return "the leap-frog substepping needs a lumped (HRZ) cut-cell mass";
    }
    if (!(out.mass[i] > 0.0)) return "a lumped cut-cell mass is not positive";
  }
  int64_t ids[kMaxN * kMaxN * kMaxN];
  for (int64_t t = 0; t < (int64_t)nd.size(); ++t) {
    const int64_t g = nd[t], r = nc + t;
    int64_t cells[8];
    int local[8];
    const int m = adjacent_cells(hs, g, cells, local);
    row.clear();
    for (int q = 0; q < m; ++q) {
      if (hs.cell_flag[cells[q]] != kUncut) return "a d node touches a cut cell";
      cell_node_ids(hs, cells[q], ids);
      const double* Ke = &hs.Ke_uncut[(size_t)local[q] * nb];
      for (int j = 0; j < nb; ++j) row.emplace_back(ids[j], Ke[j]);
      out.mass[r] += hs.Me_uncut_diag[local[q]];
    }
    // duplicates summed in a fixed order (cells as listed)
    std::stable_sort(row.begin(), row.end(),
                     [](const std::pair<int64_t, double>& a, const std::pair<int64_t, double>& b) {
                       return a.first < b.first;
                     });
    size_t o = 0;
    for (size_t k = 0; k < row.size(); ++k) {
      if (o > 0 && row[o - 1].first == row[k].first) row[o - 1].second += row[k].second;
      else row[o++] = row[k];
    }
    row.resize(o);
    push(r);
  }
  out.fx.assign(nf, 0.0);
  std::vector<int64_t> fpos(hs.n_grid, -1);
  for (int64_t r = 0; r < nf; ++r) fpos[out.node[r]] = r;
  for (size_t t = 0; t < hs.src_nodes.size(); ++t)
    if (fpos[hs.src_nodes[t]] >= 0) out.fx[fpos[hs.src_nodes[t]]] = hs.src_vals[t];
  return "";
}

}  // namespace imex
