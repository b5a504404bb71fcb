// Nested-dissection supernodal Cholesky factor of the implicit block for the
// device solve (host setup, FP64).  The method factorises S = M^cc + beta
// dt^2 K^cc once before the time loop and solves with the factor every step
// (Section "Time Integration", Newmark IMEX flowchart); this file builds that
// factor in the form the level-scheduled device kernels read: per supernode
// the inverse of its diagonal block of L and C_s = L_ts L_ss^-1 (see NdFactor
// in internal.h).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace imex {

namespace {

struct NdBuilder {
  const HostSetup& hs;
  int64_t leaf;
  std::vector<NdTreeNode>& out;

  void coords(int64_t v, int64_t* I) const {
    const int64_t g = hs.c_nodes[v];
    I[0] = g % hs.nn[0];
    I[1] = (g / hs.nn[0]) % hs.nn[1];
    I[2] = g / (hs.nn[0] * hs.nn[1]);
  }

  // Splits `rows` and appends its subtree in postorder; returns the ids of
  // the subtree's roots (more than one when a plane meets no row of a
  // disconnected set).
  std::vector<int32_t> split(std::vector<int64_t> rows) {
    const int dim = hs.dim, p = hs.p;
    if ((int64_t)rows.size() > leaf) {
      int64_t lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, hi[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
      for (int64_t v : rows) {
        int64_t I[3];
        coords(v, I);
        for (int k = 0; k < dim; ++k) {
          lo[k] = std::min(lo[k], I[k]);
          hi[k] = std::max(hi[k], I[k]);
        }
      }
      // axes by decreasing extent; the first with a cell-face plane strictly
      // inside the set is split at the plane closest to the median
      int axes[3] = {0, 1, 2};
      std::sort(axes, axes + dim, [&](int a, int b) { return hi[a] - lo[a] > hi[b] - lo[b]; });
      for (int t = 0; t < dim; ++t) {
        const int ax = axes[t];
        const int64_t first = (lo[ax] / p + 1) * p, last = ((hi[ax] - 1) / p) * p;  // planes in (lo, hi)
        if (first > last) continue;
        std::vector<int64_t> cs;
        cs.reserve(rows.size());
        for (int64_t v : rows) {
          int64_t I[3];
          coords(v, I);
          cs.push_back(I[ax]);
        }
        std::vector<int64_t> srt = cs;
        std::nth_element(srt.begin(), srt.begin() + srt.size() / 2, srt.end());
        const int64_t med = srt[srt.size() / 2];
        int64_t plane = (med + p / 2) / p * p;
        plane = std::min(std::max(plane, first), last);
        std::vector<int64_t> left, right, sep;
        for (size_t i = 0; i < rows.size(); ++i) {
          if (cs[i] < plane) left.push_back(rows[i]);
          else if (cs[i] > plane) right.push_back(rows[i]);
          else sep.push_back(rows[i]);
        }
        std::vector<int32_t> kids = split(std::move(left));
        std::vector<int32_t> r2 = split(std::move(right));
        kids.insert(kids.end(), r2.begin(), r2.end());
        if (sep.empty()) return kids;
        const int32_t id = (int32_t)out.size();
        out.emplace_back();
        out.back().rows = std::move(sep);
        for (int32_t c : kids) out[c].parent = id;
        return {id};
      }
    }
    if (rows.empty()) return {};
    const int32_t id = (int32_t)out.size();
    out.emplace_back();
    out.back().rows = std::move(rows);
    return {id};
  }
};

// ---- dense kernels on row-major blocks -------------------------------------

// In-place Cholesky of the leading m x m block of F (leading dimension ld),
// lower triangle; false on a non-positive pivot.
bool dense_cholesky(double* F, int64_t m, int64_t ld) {
  for (int64_t j = 0; j < m; ++j) {
    double* Fj = F + j * ld;
    double d = Fj[j];
    for (int64_t l = 0; l < j; ++l) d -= Fj[l] * Fj[l];
    if (!(d > 0.0)) return false;
    const double dj = std::sqrt(d);
    Fj[j] = dj;
    const double inv = 1.0 / dj;
    for (int64_t i = j + 1; i < m; ++i) {
      double* Fi = F + i * ld;
      double s = Fi[j];
      for (int64_t l = 0; l < j; ++l) s -= Fi[l] * Fj[l];
      Fi[j] = s * inv;
    }
  }
  return true;
}

}  // namespace

void nd_dissect(const HostSetup& hs, const std::vector<int64_t>& verts, int64_t leaf,
                std::vector<NdTreeNode>& out) {
  out.clear();
  NdBuilder b{hs, std::max<int64_t>(leaf, 1), out};
  b.split(verts);
  for (NdTreeNode& n : out) std::sort(n.rows.begin(), n.rows.end());
}

std::string build_nd_factor(const Csr& S, NdFactor& F, int n_threads) {
  const int64_t ns = (int64_t)F.sn.size();
  const int64_t nc = S.nrows;
  // ---- heights, structure, offsets --------------------------------------------
  std::vector<std::vector<int32_t>> children(ns);
  for (int64_t s = 0; s < ns; ++s) {
    F.sn[s].height = 0;
    if (F.sn[s].parent >= 0) {
      if (F.sn[s].parent <= s) return "nested dissection: parent before child";
      children[F.sn[s].parent].push_back((int32_t)s);
    }
  }
  for (int64_t s = 0; s < ns; ++s)
    if (F.sn[s].parent >= 0)
      F.sn[F.sn[s].parent].height = std::max(F.sn[F.sn[s].parent].height, F.sn[s].height + 1);
  std::vector<std::vector<int32_t>> st(ns);
  for (int64_t s = 0; s < ns; ++s) {
    const NdSnode& q = F.sn[s];
    const int64_t end = q.c0 + q.m;
    std::vector<int32_t>& v = st[s];
    for (int64_t i = q.c0; i < end; ++i)
      for (int64_t t = S.ptr[i]; t < S.ptr[i + 1]; ++t)
        if (S.col[t] >= end) v.push_back((int32_t)S.col[t]);
    for (int32_t c : children[s])
      for (int32_t g : st[c])
        if (g >= end) v.push_back(g);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  F.st.clear();
  F.height = -1;
  F.nnz_L = 0;
  F.max_m = F.max_mk = 0;
  int64_t off = 0, woff = 0, goff = 0;
  for (int64_t s = 0; s < ns; ++s) {
    NdSnode& q = F.sn[s];
    q.k = (int32_t)st[s].size();
    q.soff = (int64_t)F.st.size();
    F.st.insert(F.st.end(), st[s].begin(), st[s].end());
    q.foff = off;
    q.boff = off;
    off += (int64_t)q.m * (q.m + 1) / 2 + (int64_t)q.k * q.m;
    q.woff = woff;
    woff += q.k;
    q.goff = goff;
    goff += q.m + q.k;
    F.height = std::max(F.height, q.height);
    F.max_m = std::max<int64_t>(F.max_m, q.m);
    F.max_mk = std::max<int64_t>(F.max_mk, (int64_t)q.m + q.k);
  }
  F.nnz_L = off;
  F.w_len = woff;
  if (woff >= INT32_MAX) return "nested dissection: update buffer too large";
  // ---- gather slots: the children's W entries summed into b'_s and W_s ------------
  {
    std::vector<std::vector<int32_t>> src(goff);
    for (int64_t s = 0; s < ns; ++s) {
      const NdSnode& q = F.sn[s];
      for (int32_t c : children[s]) {  // fixed order: children in postorder
        const NdSnode& qc = F.sn[c];
        for (int32_t t = 0; t < qc.k; ++t) {
          const int64_t g = F.st[qc.soff + t];
          int64_t slot;
          if (g < q.c0 + q.m) {
            slot = g - q.c0;
          } else {
            const int32_t* b = F.st.data() + q.soff;
            const int32_t* e = b + q.k;
            const int32_t* it = std::lower_bound(b, e, (int32_t)g);
            if (it == e || *it != g) return "nested dissection: child structure not in the parent's";
            slot = q.m + (it - b);
          }
          src[q.goff + slot].push_back((int32_t)(qc.woff + t));
        }
      }
    }
    F.gptr.assign(goff + 1, 0);
    for (int64_t t = 0; t < goff; ++t) F.gptr[t + 1] = F.gptr[t] + (int64_t)src[t].size();
    F.gsrc.resize(F.gptr[goff]);
    for (int64_t t = 0; t < goff; ++t) std::copy(src[t].begin(), src[t].end(), F.gsrc.begin() + F.gptr[t]);
  }
  // ---- numeric factorisation (multifrontal), roots' subtrees in parallel ---------
  F.fwd.assign(off, 0.0);
  F.bwd.assign(off, 0.0);
  std::vector<int64_t> roots;
  std::vector<int64_t> sub_begin(ns);  // first supernode of each subtree (postorder)
  for (int64_t s = 0; s < ns; ++s) {
    sub_begin[s] = s;
    for (int32_t c : children[s]) sub_begin[s] = std::min(sub_begin[s], sub_begin[c]);
    if (F.sn[s].parent < 0) roots.push_back(s);
  }
  // largest subtrees first
  std::sort(roots.begin(), roots.end(), [&](int64_t a, int64_t b) {
    return a - sub_begin[a] > b - sub_begin[b];
  });
  std::vector<std::string> errs(roots.size());
#pragma omp parallel num_threads(std::max(1, n_threads))
  {
    std::vector<int64_t> fpos(nc, -1);
    std::vector<double> Fr, Xt;
    std::vector<std::vector<double>> upd(ns);  // only this thread's subtrees' entries are used
#pragma omp for schedule(dynamic, 1)
    for (int64_t ri = 0; ri < (int64_t)roots.size(); ++ri) {
      const int64_t r = roots[ri];
      for (int64_t s = sub_begin[r]; s <= r && errs[ri].empty(); ++s) {
        const NdSnode& q = F.sn[s];
        const int64_t m = q.m, k = q.k, f = m + k;
        const int32_t* sts = F.st.data() + q.soff;
        for (int64_t i = 0; i < m; ++i) fpos[q.c0 + i] = i;
        for (int64_t t = 0; t < k; ++t) fpos[sts[t]] = m + t;
        Fr.assign((size_t)(f * f), 0.0);
        // entries of S in the rows of s (columns from s on)
        for (int64_t i = 0; i < m; ++i) {
          const int64_t gi = q.c0 + i;
          for (int64_t t = S.ptr[gi]; t < S.ptr[gi + 1]; ++t) {
            const int64_t j = S.col[t];
            if (j < q.c0) continue;
            const int64_t pj = fpos[j];
            Fr[i * f + pj] = S.val[t];
            Fr[pj * f + i] = S.val[t];
          }
        }
        // extend-add of the children's update matrices
        for (int32_t c : children[s]) {
          const NdSnode& qc = F.sn[c];
          const int32_t* stc = F.st.data() + qc.soff;
          const std::vector<double>& U = upd[c];
          for (int64_t a = 0; a < qc.k; ++a) {
            const int64_t pa = fpos[stc[a]];
            for (int64_t b = 0; b < qc.k; ++b) Fr[pa * f + fpos[stc[b]]] += U[a * qc.k + b];
          }
          upd[c].clear();
          upd[c].shrink_to_fit();
        }
        for (int64_t i = 0; i < m; ++i) fpos[q.c0 + i] = -1;
        for (int64_t t = 0; t < k; ++t) fpos[sts[t]] = -1;
        // L_ss (in place), L_ts = F_ts L_ss^-T (in place)
        if (!dense_cholesky(Fr.data(), m, f)) {
          std::ostringstream os;
          os << "Cholesky factorisation of S failed (non-positive pivot) in supernode " << s;
          errs[ri] = os.str();
          break;
        }
        for (int64_t t = 0; t < k; ++t) {
          double* row = &Fr[(m + t) * f];
          for (int64_t j = 0; j < m; ++j) {
            const double* Lj = &Fr[j * f];
            double v = row[j];
            for (int64_t l = 0; l < j; ++l) v -= row[l] * Lj[l];
            row[j] = v / Lj[j];
          }
        }
        // update matrix F_tt - L_ts L_ts^T for the parent
        if (k > 0) {
          std::vector<double>& U = upd[s];
          U.assign((size_t)(k * k), 0.0);
          for (int64_t a = 0; a < k; ++a) {
            const double* La = &Fr[(m + a) * f];
            for (int64_t b = 0; b <= a; ++b) {
              const double* Lb = &Fr[(m + b) * f];
              double v = Fr[(m + a) * f + m + b];
              for (int64_t l = 0; l < m; ++l) v -= La[l] * Lb[l];
              U[a * k + b] = v;
              U[b * k + a] = v;
            }
          }
        }
        // Xt = (L_ss^-1)^T: row j is column j of the inverse, from row j on
        Xt.assign((size_t)(m * m), 0.0);
        for (int64_t j = 0; j < m; ++j) {
          double* Xj = &Xt[j * m];
          Xj[j] = 1.0 / Fr[j * f + j];
          for (int64_t i = j + 1; i < m; ++i) {
            const double* Li = &Fr[i * f];
            double v = 0.0;
            for (int64_t l = j; l < i; ++l) v -= Li[l] * Xj[l];
            Xj[i] = v / Li[i];
          }
        }
        // forward rows: L_ss^-1 row r (r + 1 values), then C_s rows (m values)
        double* fw = F.fwd.data() + q.foff;
        for (int64_t r = 0; r < m; ++r)
          for (int64_t j = 0; j <= r; ++j) fw[r * (r + 1) / 2 + j] = Xt[j * m + r];
        double* fc = fw + m * (m + 1) / 2;
        for (int64_t t = 0; t < k; ++t) {
          const double* Lt = &Fr[(m + t) * f];
          for (int64_t j = 0; j < m; ++j) {
            const double* Xj = &Xt[j * m];
            double v = 0.0;
            for (int64_t l = j; l < m; ++l) v += Lt[l] * Xj[l];
            fc[t * m + j] = v;
          }
        }
        // backward rows j: column j of L_ss^-1 from row j on, then column j of C_s
        double* bw = F.bwd.data() + q.boff;
        for (int64_t j = 0; j < m; ++j) {
          double* row = bw + j * (m + k) - j * (j - 1) / 2;
          for (int64_t i = j; i < m; ++i) row[i - j] = Xt[j * m + i];
          for (int64_t t = 0; t < k; ++t) row[m - j + t] = fc[t * m + j];
        }
      }
    }
  }
  for (const std::string& e : errs)
    if (!e.empty()) return e;
  return "";
}

void nd_solve_host(const NdFactor& F, const double* b, double* x) {
  const int64_t ns = (int64_t)F.sn.size();
  std::vector<double> W(F.w_len, 0.0), y;
  int64_t nc = 0;
  for (const NdSnode& q : F.sn) nc = std::max<int64_t>(nc, q.c0 + q.m);
  y.assign(nc, 0.0);
  std::vector<double> v;
  for (int32_t h = 0; h <= F.height; ++h)
    for (int64_t s = 0; s < ns; ++s) {
      const NdSnode& q = F.sn[s];
      if (q.height != h) continue;
      v.assign(q.m, 0.0);
      for (int32_t i = 0; i < q.m; ++i) {
        double t = b[q.c0 + i];
        for (int64_t g = F.gptr[q.goff + i]; g < F.gptr[q.goff + i + 1]; ++g) t -= W[F.gsrc[g]];
        v[i] = t;
      }
      const double* fw = F.fwd.data() + q.foff;
      for (int64_t r = 0; r < q.m + q.k; ++r) {
        const int64_t len = r < q.m ? r + 1 : q.m;
        const double* row = fw + (r < q.m ? r * (r + 1) / 2 : (int64_t)q.m * (q.m + 1) / 2 + (r - q.m) * q.m);
        double acc = 0.0;
        for (int64_t j = 0; j < len; ++j) acc += row[j] * v[j];
        if (r < q.m) {
          y[q.c0 + r] = acc;
        } else {
          for (int64_t g = F.gptr[q.goff + r]; g < F.gptr[q.goff + r + 1]; ++g) acc += W[F.gsrc[g]];
          W[q.woff + r - q.m] = acc;
        }
      }
    }
  for (int32_t h = F.height; h >= 0; --h)
    for (int64_t s = 0; s < ns; ++s) {
      const NdSnode& q = F.sn[s];
      if (q.height != h) continue;
      v.assign((size_t)q.m + q.k, 0.0);
      for (int32_t i = 0; i < q.m; ++i) v[i] = y[q.c0 + i];
      for (int32_t t = 0; t < q.k; ++t) v[q.m + t] = -x[F.st[q.soff + t]];
      const double* bw = F.bwd.data() + q.boff;
      for (int64_t j = 0; j < q.m; ++j) {
        const double* row = bw + j * (q.m + q.k) - j * (j - 1) / 2;
        const int64_t len = q.m - j + q.k;
        double acc = 0.0;
        for (int64_t t = 0; t < len; ++t) acc += row[t] * v[j + t];
        x[q.c0 + j] = acc;
      }
    }
}

}  // namespace imex
