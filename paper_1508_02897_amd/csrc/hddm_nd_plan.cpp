// Symbolic tables of the nested-dissection multifrontal local solver (the
// low-fill alternative to the line-by-line block factorisation of the local
// problems, Sec. 3).  For a box of mx x my nodes, the rectangle of a front is
// halved by a separator line across its longer side until at most `leaf`
// nodes remain, which form a leaf front.  The ring of a rectangle (the nodes
// just outside its four sides, inside the box) lies on ancestor separators, so
// it is exactly the set of later-eliminated nodes the front couples to.
#include "hddm_nd_plan.h"

#include <algorithm>
#include <functional>

namespace hddm {
namespace {

struct Rect {
  int y0, y1, x0, x1;
};

struct Tmp {
  std::vector<int> sep, bnd;
  int c0 = -1, c1 = -1, depth = 0, parent = -1;
};

int pad16(int n) { return (n + 15) / 16 * 16; }

}  // namespace

bool nd_build(const std::vector<std::pair<int, int>>& shapes, int leaf, NDPlan& pl,
              std::string& err) {
  pl = NDPlan{};
  pl.shapes = shapes;
  std::vector<std::vector<Tmp>> all(shapes.size());
  int depths = 0;
  for (size_t ci = 0; ci < shapes.size(); ++ci) {
    const int mx = shapes[ci].first, my = shapes[ci].second;
    std::vector<Tmp>& fr = all[ci];
    auto ring = [&](const Rect& r) {
      std::vector<int> b;
      if (r.y0 > 0)
        for (int x = r.x0; x < r.x1; ++x) b.push_back((r.y0 - 1) * mx + x);
      if (r.y1 < my)
        for (int x = r.x0; x < r.x1; ++x) b.push_back(r.y1 * mx + x);
      if (r.x0 > 0)
        for (int y = r.y0; y < r.y1; ++y) b.push_back(y * mx + r.x0 - 1);
      if (r.x1 < mx)
        for (int y = r.y0; y < r.y1; ++y) b.push_back(y * mx + r.x1);
      std::sort(b.begin(), b.end());
      return b;
    };
    std::function<int(Rect, int, int)> rec = [&](Rect r, int depth, int parent) -> int {
      const int h = r.y1 - r.y0, w = r.x1 - r.x0;
      if (h <= 0 || w <= 0) return -1;
      const int id = (int)fr.size();
      fr.emplace_back();
      Tmp t;
      t.depth = depth;
      t.parent = parent;
      int c0 = -1, c1 = -1;
      if (h * w <= leaf) {
        for (int y = r.y0; y < r.y1; ++y)
          for (int x = r.x0; x < r.x1; ++x) t.sep.push_back(y * mx + x);
      } else if (h >= w) {
        const int m = r.y0 + h / 2;
        for (int x = r.x0; x < r.x1; ++x) t.sep.push_back(m * mx + x);
        c0 = rec(Rect{r.y0, m, r.x0, r.x1}, depth + 1, id);
        c1 = rec(Rect{m + 1, r.y1, r.x0, r.x1}, depth + 1, id);
      } else {
        const int m = r.x0 + w / 2;
        for (int y = r.y0; y < r.y1; ++y) t.sep.push_back(y * mx + m);
        c0 = rec(Rect{r.y0, r.y1, r.x0, m}, depth + 1, id);
        c1 = rec(Rect{r.y0, r.y1, m + 1, r.x1}, depth + 1, id);
      }
      t.c0 = c0;
      t.c1 = c1;
      t.bnd = ring(r);
      fr[id] = std::move(t);
      return id;
    };
    rec(Rect{0, my, 0, mx}, 0, -1);
    for (const Tmp& t : fr) depths = std::max(depths, t.depth + 1);
  }
  pl.depths = depths;
  pl.maxcnt.assign(depths, 0);
  pl.maxn.assign(depths, 0);
  pl.maxw.assign(depths, 0);
  pl.doff.assign(shapes.size() * depths, 0);
  pl.dcnt.assign(shapes.size() * depths, 0);
  for (size_t ci = 0; ci < shapes.size(); ++ci) {
    const int mx = shapes[ci].first, my = shapes[ci].second;
    const std::vector<Tmp>& fr = all[ci];
    const int base = (int)pl.fronts.size();
    // owner of every node and its position in the owner's separator
    std::vector<int> owner(mx * my, -1), spos(mx * my, -1);
    for (int f = 0; f < (int)fr.size(); ++f)
      for (int k = 0; k < (int)fr[f].sep.size(); ++k) {
        const int g = fr[f].sep[k];
        if (owner[g] != -1) {
          err = "node on two separators";
          return false;
        }
        owner[g] = f;
        spos[g] = k;
      }
    for (int g = 0; g < mx * my; ++g)
      if (owner[g] < 0) {
        err = "node on no separator";
        return false;
      }
    auto is_desc = [&](int f, int a) {  // a is a proper descendant of f
      for (int p = fr[a].parent; p >= 0; p = fr[p].parent)
        if (p == f) return true;
      return false;
    };
    // position of node g in front f, or -1 if g is not in f's separator or ring
    auto fpos = [&](int f, int g) {
      const Tmp& t = fr[f];
      if (owner[g] == f) return spos[g];
      auto it = std::lower_bound(t.bnd.begin(), t.bnd.end(), g);
      if (it != t.bnd.end() && *it == g) return pad16((int)t.sep.size()) + (int)(it - t.bnd.begin());
      return -1;
    };
    std::vector<int64_t> usum(depths, 0), vsum(depths, 0);
    int64_t gsum = 0;
    std::vector<NDFront> out(fr.size());
    for (int f = 0; f < (int)fr.size(); ++f) {
      const Tmp& t = fr[f];
      NDFront& o = out[f];
      o.s = (int)t.sep.size();
      o.b = (int)t.bnd.size();
      o.sp = pad16(o.s);
      o.bp = pad16(o.b);
      o.depth = t.depth;
      if (o.sp + o.bp > ND_MAX_N || o.s + o.b > ND_MAX_W) {
        err = "front of " + std::to_string(o.s) + " + " + std::to_string(o.b) + " nodes is too large";
        return false;
      }
      o.node_off = (int)pl.nodes.size();
      pl.nodes.insert(pl.nodes.end(), t.sep.begin(), t.sep.end());
      pl.nodes.insert(pl.nodes.end(), t.bnd.begin(), t.bnd.end());
      o.asm_off = (int)pl.asmp.size();
      for (int g : t.sep) {
        const int j = g / mx, x = g - j * mx;
        const int nb[4] = {x > 0 ? g - 1 : -1, x + 1 < mx ? g + 1 : -1, j > 0 ? g - mx : -1,
                           j + 1 < my ? g + mx : -1};
        for (int q = 0; q < 4; ++q) {
          int pos = -1;
          if (nb[q] >= 0) {
            pos = fpos(f, nb[q]);
            // a neighbour outside the front must have been eliminated below
            if (pos < 0 && !is_desc(f, owner[nb[q]])) {
              err = "neighbour neither in the front nor below it";
              return false;
            }
          }
          pl.asmp.push_back(pos);
        }
      }
      o.c0 = t.c0 < 0 ? -1 : base + t.c0;
      o.c1 = t.c1 < 0 ? -1 : base + t.c1;
      const int cs[2] = {t.c0, t.c1};
      int* cm[2] = {&o.cmap0, &o.cmap1};
      for (int q = 0; q < 2; ++q) {
        *cm[q] = (int)pl.cmap.size();
        if (cs[q] < 0) continue;
        if (fr[cs[q]].depth != t.depth + 1) {
          err = "child depth";
          return false;
        }
        for (int g : fr[cs[q]].bnd) {
          const int pos = fpos(f, g);
          if (pos < 0) {
            err = "child ring node missing from the parent front";
            return false;
          }
          pl.cmap.push_back(pos);
        }
      }
      o.g_off = (int32_t)gsum;
      gsum += (int64_t)o.s * o.s + 2 * (int64_t)o.b * o.s;
      o.u_off = (int32_t)usum[t.depth];
      usum[t.depth] += (int64_t)o.b * o.b;
      o.v_off = (int32_t)vsum[t.depth];
      vsum[t.depth] += (int64_t)o.b * BLOCK_RHS;
      pl.maxn[t.depth] = std::max(pl.maxn[t.depth], o.sp + o.bp);
      pl.maxw[t.depth] = std::max(pl.maxw[t.depth], o.s + o.b);
      // front matrix and the three 16-row Gauss-Jordan panels
      const int64_t nn = o.sp + o.bp;
      pl.wstride = std::max(pl.wstride, nn * nn + 3 * 16 * nn);
    }
    if (gsum > INT32_MAX) {
      err = "box factor too large";
      return false;
    }
    pl.class_entries.push_back((gsum + 31) & ~int64_t(31));
    for (int d = 0; d < depths; ++d) {
      pl.ustride = std::max(pl.ustride, (usum[d] + 31) & ~int64_t(31));
      pl.vstride = std::max(pl.vstride, (vsum[d] + 31) & ~int64_t(31));
    }
    pl.fronts.insert(pl.fronts.end(), out.begin(), out.end());
    for (int d = 0; d < depths; ++d) {
      pl.doff[ci * depths + d] = (int)pl.dlist.size();
      int cnt = 0;
      for (int f = 0; f < (int)fr.size(); ++f)
        if (fr[f].depth == d) {
          pl.dlist.push_back(base + f);
          ++cnt;
        }
      pl.dcnt[ci * depths + d] = cnt;
      pl.maxcnt[d] = std::max(pl.maxcnt[d], cnt);
    }
  }
  pl.wstride = (pl.wstride + 31) & ~int64_t(31);
  // every position the kernels use lies inside its front
  for (const NDFront& o : pl.fronts) {
    for (int k = 0; k < 4 * o.s; ++k) {
      const int p = pl.asmp[o.asm_off + k];
      if (p < -1 || p >= o.sp + o.bp || (p >= o.s && p < o.sp)) {
        err = "assembly position out of range";
        return false;
      }
    }
    const int cs[2] = {o.c0, o.c1}, cm[2] = {o.cmap0, o.cmap1};
    for (int q = 0; q < 2; ++q) {
      if (cs[q] < 0) continue;
      for (int p = 0; p < pl.fronts[cs[q]].b; ++p) {
        const int v = pl.cmap[cm[q] + p];
        if (v < 0 || v >= o.sp + o.bp || (v >= o.s && v < o.sp)) {
          err = "child map out of range";
          return false;
        }
      }
    }
  }
  return true;
}

}  // namespace hddm
