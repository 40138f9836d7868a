// Host planner: label classification, mode grouping and fusion, orientation,
// gather directions and block-scatter indexing vectors.
//
// The paper's block-scatter mapping (Approach, "Supporting tensor
// computations") views a tensor as a matrix through per-row and per-column
// offset vectors, so matrix code runs on the tensor with one extra level of
// indirection and no tensor is ever transposed in memory (Approach,
// "Variations on functionality": transposition by exchanging strides).  The
// partitioning of the three index groups is conformal across the operands
// that share them (Approach, "Flexible abstractions", footnote on C = AB).
#include <algorithm>
#include <cstdlib>
#include <limits>

#include "internal.hpp"

namespace famlies {

namespace {

inline int64_t iabs(int64_t v) { return v < 0 ? -v : v; }

bool check_tensor(const famlies_tensor* t, const char* name, std::string* err) {
  if (!t) {
    *err = std::string(name) + ": null descriptor";
    return false;
  }
  if (t->rank < 0 || t->rank > FAMLIES_MAX_RANK) {
    *err = std::string(name) + ": rank out of range [0, 8]";
    return false;
  }
  if (t->rank > 0 && (!t->extents || !t->strides || !t->labels)) {
    *err = std::string(name) + ": null extents/strides/labels";
    return false;
  }
  for (int d = 0; d < t->rank; ++d) {
    if (t->extents[d] < 0) {
      *err = std::string(name) + ": negative extent";
      return false;
    }
  }
  return true;
}

bool repeated(const famlies_tensor* t) {
  for (int d = 0; d < t->rank; ++d)
    for (int e = 0; e < d; ++e)
      if (t->labels[d] == t->labels[e]) return true;
  return false;
}

// [lo, hi] of element offsets; lo > hi when the tensor has no elements.
void span(const famlies_tensor* t, int64_t* lo, int64_t* hi) {
  int64_t l = 0, h = 0;
  for (int d = 0; d < t->rank; ++d) {
    if (t->extents[d] == 0) {
      *lo = 0;
      *hi = -1;
      return;
    }
    int64_t r = (t->extents[d] - 1) * t->strides[d];
    if (r < 0) l += r; else h += r;
  }
  *lo = l;
  *hi = h;
}

// Sufficient condition for an injective layout: with modes of extent > 1
// sorted by |stride|, every |stride| exceeds the largest offset reachable by
// the smaller modes.
bool injective(const famlies_tensor* t) {
  std::vector<std::pair<int64_t, int64_t>> m;  // (|stride|, extent)
  for (int d = 0; d < t->rank; ++d) {
    if (t->extents[d] == 0) return true;  // no elements at all
    if (t->extents[d] > 1) m.push_back({iabs(t->strides[d]), t->extents[d]});
  }
  std::sort(m.begin(), m.end());
  int64_t reach = 0;
  for (auto& s : m) {
    if (s.first <= reach) return false;
    reach += (s.second - 1) * s.first;
  }
  return true;
}

int64_t sel(const Mode& md, int which) { return which == 0 ? md.sx : which == 1 ? md.sy : md.sc; }

// Fuse neighbours u, v (in group order) when, in every operand holding the
// group, v's stride equals u's extent times u's stride: the pair then walks
// memory exactly like one mode of extent e_u * e_v.
std::vector<Mode> fuse(const std::vector<Mode>& in, int w1, int w2) {
  std::vector<Mode> out;
  for (const Mode& md : in) {
    if (!out.empty()) {
      Mode& u = out.back();
      if (sel(md, w1) == u.ext * sel(u, w1) && sel(md, w2) == u.ext * sel(u, w2)) {
        u.ext *= md.ext;
        continue;
      }
    }
    out.push_back(md);
  }
  return out;
}

int64_t min_abs(const std::vector<Mode>& g, int which) {
  int64_t m = std::numeric_limits<int64_t>::max();
  for (const Mode& md : g) m = std::min(m, iabs(sel(md, which)));
  return m;
}

int64_t reach(const std::vector<Mode>& g, int which) {
  int64_t r = 0;
  for (const Mode& md : g) r += (md.ext - 1) * iabs(sel(md, which));
  return r;
}

// Sum over the modes of the most negative offset each can contribute.
int64_t lowest(const std::vector<Mode>& g, int which) {
  int64_t r = 0;
  for (const Mode& md : g) {
    const int64_t t = (md.ext - 1) * sel(md, which);
    if (t < 0) r += t;
  }
  return r;
}

}  // namespace

int analyze(int dtype, int compute, const famlies_tensor* A, const famlies_tensor* B,
            const famlies_tensor* C, Analysis* out, std::string* err) {
  if (dtype != FAMLIES_F64 && dtype != FAMLIES_F32) {
    *err = "dtype must be FAMLIES_F64 or FAMLIES_F32";
    return FAMLIES_ERR_INVALID_ARG;
  }
  const bool int8 = compute >= FAMLIES_INT8X3 && compute <= FAMLIES_INT8X7;
  if (compute != FAMLIES_NATIVE && compute != FAMLIES_BF16X3 && compute != FAMLIES_BF16X6 && !int8) {
    *err = "compute must be FAMLIES_NATIVE, FAMLIES_BF16X3, FAMLIES_BF16X6 or FAMLIES_INT8X3..FAMLIES_INT8X7";
    return FAMLIES_ERR_INVALID_ARG;
  }
  if ((compute == FAMLIES_BF16X3 || compute == FAMLIES_BF16X6) && dtype != FAMLIES_F32) {
    *err = "split-bf16 compute needs FAMLIES_F32 data";
    return FAMLIES_ERR_UNSUPPORTED;
  }
  if (int8 && dtype != FAMLIES_F64) {
    *err = "FP64 emulation on INT8 needs FAMLIES_F64 data";
    return FAMLIES_ERR_UNSUPPORTED;
  }
  if (!check_tensor(A, "A", err) || !check_tensor(B, "B", err) || !check_tensor(C, "C", err))
    return FAMLIES_ERR_INVALID_ARG;
  if (repeated(C)) {
    *err = "a label is repeated within C";
    return FAMLIES_ERR_LABEL;
  }
  Analysis an;
  an.dtype = dtype;
  an.compute = compute;
  an.esize = dtype == FAMLIES_F64 ? 8 : 4;
  // Distinct labels with their extent and summed stride in each tensor
  // (summing the strides of a repeated label addresses its diagonal).
  struct Lab {
    int32_t label;
    int64_t ext;
    int64_t s[3];
    int cnt[3];
  };
  std::vector<Lab> labs;
  const famlies_tensor* T3[3] = {A, B, C};
  for (int t = 0; t < 3; ++t) {
    for (int d = 0; d < T3[t]->rank; ++d) {
      const int32_t l = T3[t]->labels[d];
      const int64_t e = T3[t]->extents[d];
      Lab* f = nullptr;
      for (Lab& x : labs)
        if (x.label == l) f = &x;
      if (!f) {
        labs.push_back({l, e, {0, 0, 0}, {0, 0, 0}});
        f = &labs.back();
      } else if (f->ext != e) {
        *err = "one label has two different extents";
        return FAMLIES_ERR_SHAPE_MISMATCH;
      }
      f->s[t] += T3[t]->strides[d];
      f->cnt[t] += 1;
    }
  }
  std::vector<Mode> I, J, P, Lm;  // in user orientation: sx = A stride, sy = B stride
  for (const Lab& x : labs) {
    const bool a = x.cnt[0] > 0, b = x.cnt[1] > 0, c = x.cnt[2] > 0;
    if (x.cnt[0] > 1 || x.cnt[1] > 1) an.n_diag++;
    Mode m{x.label, x.ext, x.s[0], x.s[1], x.s[2]};
    if (c && !a && !b) {
      *err = "a label of C appears in neither A nor B";
      return FAMLIES_ERR_LABEL;
    }
    if (a && b && c)
      Lm.push_back(m);
    else if (a && c)
      I.push_back(m);
    else if (b && c)
      J.push_back(m);
    else {
      if (!(a && b)) an.n_trace++;  // summed inside one input: zero stride in the other
      P.push_back(m);
    }
  }
  if (!injective(C)) {
    *err = "C's layout maps two multi-indices to one address";
    return FAMLIES_ERR_ALIAS;
  }
  span(A, &an.a_lo, &an.a_hi);
  span(B, &an.b_lo, &an.b_hi);
  span(C, &an.c_lo, &an.c_hi);

  auto prod = [](const std::vector<Mode>& g) {
    int64_t p = 1;
    for (const Mode& m : g) p *= m.ext;
    return p;
  };
  int64_t M = prod(I), N = prod(J), K = prod(P), L = prod(Lm);

  // Drop extent-1 modes (offset always 0).  Extent-0 modes stay so the
  // products remain 0; such problems never reach a kernel.
  auto drop1 = [](std::vector<Mode>& g) {
    g.erase(std::remove_if(g.begin(), g.end(), [](const Mode& m) { return m.ext == 1; }), g.end());
  };
  drop1(I);
  drop1(J);
  drop1(P);
  drop1(Lm);

  // Orientation and mode order.  The kernel gathers its X operand along rows
  // or along K, Y along columns or along K, taking per operand the direction
  // whose first mode has the smaller stride, and writes C with lanes along
  // its columns (the MFMA lane index).  A direction whose first mode has unit
  // stride is coalesced; a stride of s elements spreads a wave's accesses
  // over about s times as many cache lines (counted up to 16).  Per output
  // element and 128 x 128 tile, X and Y each move K/128 elements and C two
  // (read and write), so a choice costs
  //     K/128 * (cost_X + cost_Y) + 2 * cost_C,
  // minimised over the orientation (C = A B or C^T = B^T A^T) and, per group,
  // the operand whose strides order it (rows: C or X, columns: C or Y,
  // contracted: X or Y).  The default (C's smallest stride along the
  // columns, rows and columns in C's order, contracted modes in the order of
  // the operand with the smaller contracted stride) wins ties.
  auto by = [](int w1, int w2) {
    return [w1, w2](const Mode& a, const Mode& b) {
      int64_t x = iabs(sel(a, w1)), y = iabs(sel(b, w1));
      if (x != y) return x < y;
      return iabs(sel(a, w2)) < iabs(sel(b, w2));
    };
  };
  auto first = [](const std::vector<Mode>& g, int which) {
    return g.empty() ? std::numeric_limits<int64_t>::max() : iabs(sel(g.front(), which));
  };
  // cost of gathering one operand: the better of its two directions
  auto gather_cost = [&](const std::vector<Mode>& free, const std::vector<Mode>& con, int which) {
    const int64_t st = std::min(first(free, which), first(con, which));
    return (double)std::min<int64_t>(std::max<int64_t>(st, 1), 16);
  };
  struct Choice {
    bool swapped;
    std::vector<Mode> I, J, P;
    double cost;
  };
  auto evaluate = [&](bool swp, int io, int jo, int po) {
    Choice ch{swp, I, J, P, 0.0};
    if (swp) {
      std::swap(ch.I, ch.J);
      for (Mode& m : ch.I) std::swap(m.sx, m.sy);
      for (Mode& m : ch.J) std::swap(m.sx, m.sy);
      for (Mode& m : ch.P) std::swap(m.sx, m.sy);
    }
    std::stable_sort(ch.I.begin(), ch.I.end(), io == 0 ? by(2, 0) : by(0, 2));
    std::stable_sort(ch.J.begin(), ch.J.end(), jo == 0 ? by(2, 1) : by(1, 2));
    if (po < 0) po = min_abs(ch.P, 0) <= min_abs(ch.P, 1) ? 0 : 1;
    std::stable_sort(ch.P.begin(), ch.P.end(), po == 0 ? by(0, 1) : by(1, 0));
    const double cx = gather_cost(ch.I, ch.P, 0), cy = gather_cost(ch.J, ch.P, 1);
    const double cc = ch.J.empty() ? 1.0 : gather_cost(ch.J, {}, 2);
    ch.cost = (double)K / 128.0 * (cx + cy) + 2.0 * cc;
    return ch;
  };
  const bool swap0 = !I.empty() && min_abs(I, 2) < min_abs(J, 2);
  Choice best = evaluate(swap0, 0, 0, -1);
  for (int swp = 0; swp < 2; ++swp)
    for (int io = 0; io < 2; ++io)
      for (int jo = 0; jo < 2; ++jo)
        for (int po = 0; po < 2; ++po) {
          Choice ch = evaluate(swp != 0, io, jo, po);
          if (ch.cost < best.cost * (1.0 - 1e-9)) best = std::move(ch);
        }
  an.swapped = best.swapped;
  if (an.swapped) {
    std::swap(M, N);
    for (Mode& m : Lm) std::swap(m.sx, m.sy);
  }
  an.I = fuse(best.I, 0, 2);
  an.J = fuse(best.J, 1, 2);
  an.P = fuse(best.P, 0, 1);
  std::stable_sort(Lm.begin(), Lm.end(), by(2, 0));
  an.Lm = Lm;  // batch modes: not fused (one offset per batch index in each operand)
  an.M = M;
  an.N = N;
  an.K = K;
  an.L = L;

  // Gather direction per operand: along the contracted modes unless the free
  // group's first mode has a strictly smaller stride (ties go to K, the
  // LDS-contiguous way; an empty free group has no rows to gather along).
  an.x_kfast = !an.P.empty() && first(an.P, 0) <= first(an.I, 0);
  an.y_kfast = !an.P.empty() && first(an.P, 1) <= first(an.J, 1);

  // Both operands gathered along K but fastest along different contracted
  // modes u (of X) and w (of Y): a K slice in plain order would be one run
  // for X and single elements for Y.  Enumerate K instead in bu x bw blocks
  // of (u, w), so one slice holds runs of bu consecutive X elements and of bw
  // consecutive Y elements.  The K order is shared by X and Y, so any such
  // enumeration is valid.
  if (an.P.size() >= 2) {
    size_t iu = 0, iw = 0;
    for (size_t q = 1; q < an.P.size(); ++q) {
      if (iabs(an.P[q].sx) < iabs(an.P[iu].sx)) iu = q;
      if (iabs(an.P[q].sy) < iabs(an.P[iw].sy)) iw = q;
    }
    const int64_t su = iabs(an.P[iu].sx), sw = iabs(an.P[iw].sy);
    if (iu != iw && su >= 1 && su <= 2 && sw >= 1 && sw <= 2 && su <= first(an.I, 0) && sw <= first(an.J, 1)) {
      std::vector<Mode> q{an.P[iu], an.P[iw]};
      for (size_t r = 0; r < an.P.size(); ++r)
        if (r != iu && r != iw) q.push_back(an.P[r]);
      const int64_t bk = an.esize == 8 ? 8 : 32;  // the plain kernels' K slice
      q[0].blk = std::min<int64_t>(q[0].ext, bk == 32 ? 8 : 4);
      q[1].blk = std::max<int64_t>(1, std::min<int64_t>(q[1].ext, bk / q[0].blk));
      an.P = q;
      an.x_kfast = an.y_kfast = true;
    }
  }
  an.max_abs_x = reach(an.I, 0) + reach(an.P, 0) + reach(an.Lm, 0);
  an.max_abs_y = reach(an.J, 1) + reach(an.P, 1) + reach(an.Lm, 1);
  an.max_abs_c = reach(an.I, 2) + reach(an.J, 2) + reach(an.Lm, 2);
  an.x_lo = lowest(an.I, 0) + lowest(an.P, 0);
  an.y_lo = lowest(an.J, 1) + lowest(an.P, 1);
  an.c_lo_mn = lowest(an.I, 2) + lowest(an.J, 2);
  an.x_span = reach(an.I, 0) + reach(an.P, 0);
  an.y_span = reach(an.J, 1) + reach(an.P, 1);
  an.c_span = reach(an.I, 2) + reach(an.J, 2);
  *out = an;
  return FAMLIES_OK;
}

void offsets(const std::vector<Mode>& modes, int which, int64_t n, int64_t n_pad,
             std::vector<int64_t>& out) {
  out.assign(static_cast<size_t>(n_pad), 0);
  if (modes.size() >= 2 && modes[0].blk > 0 && modes[1].blk > 0) {
    // blocked: (u in block, w in block, u block, w block, remaining modes)
    const Mode& u = modes[0];
    const Mode& w = modes[1];
    const std::vector<Mode> rest(modes.begin() + 2, modes.end());
    std::vector<int64_t> outer;
    int64_t nrest = 1;
    for (const Mode& m : rest) nrest *= m.ext;
    offsets(rest, which, nrest, nrest, outer);
    const int64_t su = sel(u, which), sw = sel(w, which);
    int64_t i = 0;
    for (int64_t r = 0; r < nrest && i < n; ++r)
      for (int64_t w0 = 0; w0 < w.ext && i < n; w0 += w.blk)
        for (int64_t u0 = 0; u0 < u.ext && i < n; u0 += u.blk)
          for (int64_t b = w0; b < std::min(w.ext, w0 + w.blk) && i < n; ++b)
            for (int64_t a = u0; a < std::min(u.ext, u0 + u.blk) && i < n; ++a)
              out[static_cast<size_t>(i++)] = outer[static_cast<size_t>(r)] + a * su + b * sw;
    return;
  }
  std::vector<int64_t> digit(modes.size(), 0);
  int64_t off = 0;
  for (int64_t i = 0; i < n; ++i) {
    out[static_cast<size_t>(i)] = off;
    for (size_t d = 0; d < modes.size(); ++d) {
      int64_t s = sel(modes[d], which);
      if (++digit[d] < modes[d].ext) {
        off += s;
        break;
      }
      off -= (modes[d].ext - 1) * s;
      digit[d] = 0;
    }
  }
}

bool offsets_in_span(const std::vector<int64_t>& a, int64_t na, const std::vector<int64_t>& b, int64_t nb,
                     const std::vector<int64_t>& l, int64_t nl, int64_t lo, int64_t hi) {
  if (na <= 0 || nb <= 0 || nl <= 0) return true;  // no element is addressed
  if ((int64_t)a.size() < na || (int64_t)b.size() < nb || (int64_t)l.size() < nl || lo > hi) return false;
  auto ext = [](const std::vector<int64_t>& v, int64_t n, int64_t* mn, int64_t* mx) {
    *mn = *mx = v[0];
    for (int64_t i = 1; i < n; ++i) {
      *mn = std::min(*mn, v[(size_t)i]);
      *mx = std::max(*mx, v[(size_t)i]);
    }
  };
  int64_t a0, a1, b0, b1, l0, l1;
  ext(a, na, &a0, &a1);
  ext(b, nb, &b0, &b1);
  ext(l, nl, &l0, &l1);
  // |offsets| are bounded by the spans checked in analyze(), far below 2^62
  return a0 + b0 + l0 >= lo && a1 + b1 + l1 <= hi;
}

}  // namespace famlies
