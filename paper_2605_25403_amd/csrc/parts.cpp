// Row partition of the P1-P1 pattern for the one-kernel-per-iteration CG of
// the pressure Poisson system (kernels_fcg.hip).
//
// Parts are sets of at most rows_max rows found by recursive coordinate
// bisection of the DOF coordinates (each cut halves the part count along the
// longest extent, with sizes in proportion), so a part is a compact patch and
// its halo (the columns its rows reference outside it) is its perimeter. Rows
// are renumbered so that each part is contiguous ("part order"; inside a part
// the original order is kept). Each part stores its rows in SELL-64 slices of
// its own, whose column indices are local: 0 .. own-1 for the part's rows,
// own .. own+nhalo-1 for its halo in the order of halo[]. Padding entries
// repeat the row's last local column and take value 0.
#include <algorithm>
#include <mutex>
#include <numeric>

#include "common.hpp"
#include "mesh.hpp"

namespace ipcs {

namespace {

void rcb(std::vector<int32_t>& idx, size_t lo, size_t hi, int64_t k, const double* X, int dim,
         std::vector<int32_t>& sizes) {
  if (k == 1) {
    sizes.push_back((int32_t)(hi - lo));
    return;
  }
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (size_t q = lo; q < hi; ++q)
    for (int a = 0; a < dim; ++a) {
      const double v = X[(size_t)idx[q] * dim + a];
      mn[a] = std::min(mn[a], v);
      mx[a] = std::max(mx[a], v);
    }
  int ax = 0;
  for (int a = 1; a < dim; ++a)
    if (mx[a] - mn[a] > mx[ax] - mn[ax]) ax = a;
  const int64_t k1 = k / 2;
  const size_t n = hi - lo;
  const size_t n1 = (size_t)((n * (size_t)k1 + (size_t)k / 2) / (size_t)k);
  std::nth_element(idx.begin() + lo, idx.begin() + lo + n1, idx.begin() + hi,
                   [&](int32_t a, int32_t b) {
                     const double xa = X[(size_t)a * dim + ax], xb = X[(size_t)b * dim + ax];
                     return xa < xb || (xa == xb && a < b);
                   });
  rcb(idx, lo, lo + n1, k1, X, dim, sizes);
  rcb(idx, lo + n1, hi, k - k1, X, dim, sizes);
}

// The second halo ring of every part and the SELL-64 slices of its halo rows
// (two CG iterations per launch: a block forms B p on its own and halo rows,
// which read p on the second ring too).
void build_second_ring(const Pattern& P, const Sell& S, const std::vector<int32_t>& iperm,
                       PartSell& R) {
  R.halo2_ptr.assign(R.nparts + 1, 0);
  R.hslice_ptr.assign(R.nparts + 1, 0);
  R.hsptr.assign(1, 0);
  R.halo2.clear();
  R.hlcol.clear();
  R.hsrc.clear();
  R.lds2_max = 0;
  std::vector<int32_t> h2;
  for (int p = 0; p < R.nparts; ++p) {
    const int32_t p0 = R.part_ptr[p], p1 = R.part_ptr[p + 1], own = p1 - p0;
    const int32_t* hb = R.halo.data() + R.halo_ptr[p];
    const int32_t* he = R.halo.data() + R.halo_ptr[p + 1];
    const int nh = (int)(he - hb);
    auto in_halo = [&](int32_t c) { return std::binary_search(hb, he, c); };
    h2.clear();
    for (const int32_t* hp = hb; hp != he; ++hp) {
      const int32_t o = R.perm[*hp];
      for (int32_t q = P.rowptr[o]; q < P.rowptr[o + 1]; ++q) {
        const int32_t c = iperm[P.col[q]];
        if ((c < p0 || c >= p1) && !in_halo(c)) h2.push_back(c);
      }
    }
    std::sort(h2.begin(), h2.end());
    h2.erase(std::unique(h2.begin(), h2.end()), h2.end());
    const int64_t local = (int64_t)own + nh + (int64_t)h2.size();
    if (local > 65535) fail(IPCS_E_CAPACITY, "a part's two halo rings reference too many rows");
    R.lds2_max = std::max<int>(R.lds2_max, (int)local);
    R.halo2.insert(R.halo2.end(), h2.begin(), h2.end());
    R.halo2_ptr[p + 1] = (int32_t)R.halo2.size();
    auto loc = [&](int32_t c) -> uint16_t {
      if (c >= p0 && c < p1) return (uint16_t)(c - p0);
      const int32_t* f = std::lower_bound(hb, he, c);
      if (f != he && *f == c) return (uint16_t)(own + (f - hb));
      return (uint16_t)(own + nh + (std::lower_bound(h2.begin(), h2.end(), c) - h2.begin()));
    };
    const int nsl = (nh + 63) / 64;
    for (int sl = 0; sl < nsl; ++sl) {
      int w = 0;
      for (int lane = 0; lane < 64; ++lane) {
        const int q = 64 * sl + lane;
        if (q < nh) w = std::max(w, P.rowptr[R.perm[hb[q]] + 1] - P.rowptr[R.perm[hb[q]]]);
      }
      const int64_t base = R.hsptr.back();
      if (base + 64ll * w >= (int64_t(1) << 31)) fail(IPCS_E_CAPACITY, "partition too large");
      R.hlcol.resize(base + 64ll * w);
      R.hsrc.resize(base + 64ll * w);
      for (int lane = 0; lane < 64; ++lane) {
        const int q = 64 * sl + lane;
        const int32_t o = q < nh ? R.perm[hb[q]] : -1;
        const int len = o >= 0 ? P.rowptr[o + 1] - P.rowptr[o] : 0;
        uint16_t last = o >= 0 ? (uint16_t)(own + q) : 0;
        for (int k = 0; k < w; ++k) {
          const int64_t e = base + 64ll * k + lane;
          if (k < len) {
            last = loc(iperm[P.col[P.rowptr[o] + k]]);
            R.hlcol[e] = last;
            R.hsrc[e] = (int32_t)S.index(o, k);
          } else {
            R.hlcol[e] = last;
            R.hsrc[e] = -1;
          }
        }
      }
      R.hsptr.push_back((int32_t)(base + 64ll * w));
    }
    R.hslice_ptr[p + 1] = R.hslice_ptr[p] + nsl;
  }
  R.hnent = R.hsptr.back();
}

}  // namespace

std::shared_ptr<const PartSell> build_parts(const Pattern& P, const Sell& S, const double* X,
                                            int dim, int rows_max, int depth) {
  if (P.nrows != P.ncols) fail(IPCS_E_INVALID, "partition of a non-square pattern");
  if (depth != 1 && depth != 2) fail(IPCS_E_INVALID, "partition halo depth must be 1 or 2");
  if (rows_max < 64 || rows_max > 4096)
    fail(IPCS_E_INVALID, "rows per part must be in [64, 4096]");
  auto out = std::make_shared<PartSell>();
  PartSell& R = *out;
  const int64_t n = P.nrows;
  R.n = n;
  R.rows_max = rows_max;
  // part count: the least for which every part fits
  std::vector<int32_t> idx(n), sizes;
  for (int64_t k = std::max<int64_t>(1, div_up(n, (int64_t)rows_max));; ++k) {
    std::iota(idx.begin(), idx.end(), 0);
    sizes.clear();
    rcb(idx, 0, (size_t)n, k, X, dim, sizes);
    if (*std::max_element(sizes.begin(), sizes.end()) <= rows_max) break;
  }
  R.nparts = (int)sizes.size();
  R.part_ptr.assign(R.nparts + 1, 0);
  for (int p = 0; p < R.nparts; ++p) R.part_ptr[p + 1] = R.part_ptr[p] + sizes[p];
  for (int p = 0; p < R.nparts; ++p)
    std::sort(idx.begin() + R.part_ptr[p], idx.begin() + R.part_ptr[p + 1]);
  R.perm = idx;
  std::vector<int32_t> iperm(n);
  for (int64_t i = 0; i < n; ++i) iperm[R.perm[i]] = (int32_t)i;

  // halos and per-part SELL-64 slices with local columns
  R.halo_ptr.assign(R.nparts + 1, 0);
  R.slice_ptr.assign(R.nparts + 1, 0);
  R.sptr.assign(1, 0);
  R.maxw = 0;
  R.lds_max = 0;
  std::vector<int32_t> h;
  for (int p = 0; p < R.nparts; ++p) {
    const int32_t p0 = R.part_ptr[p], p1 = R.part_ptr[p + 1], own = p1 - p0;
    h.clear();
    for (int32_t i = p0; i < p1; ++i) {
      const int32_t o = R.perm[i];
      for (int32_t q = P.rowptr[o]; q < P.rowptr[o + 1]; ++q) {
        const int32_t c = iperm[P.col[q]];
        if (c < p0 || c >= p1) h.push_back(c);
      }
    }
    std::sort(h.begin(), h.end());
    h.erase(std::unique(h.begin(), h.end()), h.end());
    const int64_t local = (int64_t)own + (int64_t)h.size();
    if (local > 65535) fail(IPCS_E_CAPACITY, "a part references too many columns");
    R.lds_max = std::max<int>(R.lds_max, (int)local);
    R.halo.insert(R.halo.end(), h.begin(), h.end());
    R.halo_ptr[p + 1] = (int32_t)R.halo.size();
    auto loc = [&](int32_t c) -> uint16_t {
      if (c >= p0 && c < p1) return (uint16_t)(c - p0);
      return (uint16_t)(own + (std::lower_bound(h.begin(), h.end(), c) - h.begin()));
    };
    const int nsl = (own + 63) / 64;
    for (int sl = 0; sl < nsl; ++sl) {
      int w = 0;
      for (int lane = 0; lane < 64; ++lane) {
        const int32_t i = p0 + 64 * sl + lane;
        if (i < p1) w = std::max(w, P.rowptr[R.perm[i] + 1] - P.rowptr[R.perm[i]]);
      }
      R.maxw = std::max(R.maxw, w);
      const int64_t base = R.sptr.back();
      if (base + 64ll * w >= (int64_t(1) << 31)) fail(IPCS_E_CAPACITY, "partition too large");
      R.lcol.resize(base + 64ll * w);
      R.src.resize(base + 64ll * w);
      for (int lane = 0; lane < 64; ++lane) {
        const int32_t i = p0 + 64 * sl + lane;
        const int32_t o = i < p1 ? R.perm[i] : -1;
        const int len = o >= 0 ? P.rowptr[o + 1] - P.rowptr[o] : 0;
        uint16_t last = o >= 0 ? (uint16_t)(i - p0) : 0;
        for (int k = 0; k < w; ++k) {
          const int64_t e = base + 64ll * k + lane;
          if (k < len) {
            last = loc(iperm[P.col[P.rowptr[o] + k]]);
            R.lcol[e] = last;
            R.src[e] = (int32_t)S.index(o, k);
          } else {
            R.lcol[e] = last;
            R.src[e] = -1;
          }
        }
      }
      R.sptr.push_back((int32_t)(base + 64ll * w));
    }
    R.slice_ptr[p + 1] = R.slice_ptr[p] + nsl;
  }
  R.nent = R.sptr.back();
  R.depth = depth;
  if (depth == 2) build_second_ring(P, S, iperm, R);
  return out;
}

std::shared_ptr<const PartSell> Mesh::parts11(int rows_max, int depth) const {
  std::lock_guard<std::mutex> lk(parts_mu);
  for (auto& q : parts_cache)
    if (q->rows_max == rows_max && q->depth == depth) return q;
  auto q = build_parts(p11, e11, xp.data(), dim, rows_max, depth);
  parts_cache.push_back(q);
  return q;
}

}  // namespace ipcs
