// Host side of the nested-dissection local solver: the symbolic tables of the
// multifrontal factorisation for every distinct box shape.
#pragma once

#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "hddm_internal.h"

namespace hddm {

struct NDPlan {
  // one class per distinct box shape (mx, my)
  std::vector<std::pair<int, int>> shapes;
  std::vector<NDFront> fronts;   // all classes, concatenated
  std::vector<int32_t> nodes, asmp, cmap;
  std::vector<int32_t> dlist, doff, dcnt;  // per class and depth
  std::vector<int64_t> class_entries;      // factor entries of one box of the class
  int depths = 0;
  int64_t ustride = 0, vstride = 0;        // per box and depth parity (entries)
  int64_t wstride = 0;                     // one factor working matrix and its
                                           // Gauss-Jordan panels (entries)
  std::vector<int> maxcnt, maxn, maxw;     // per depth: most fronts of a class, largest
                                           // padded front (sp + bp), largest front (s + b)
};

// Build the tables for these box shapes; leaf: largest leaf rectangle (nodes).
// Checks every index the kernels form from the tables (front positions, node
// indices, child maps, stack offsets) and returns false with a message if one
// is out of range or a front exceeds ND_MAX_N / ND_MAX_W.
bool nd_build(const std::vector<std::pair<int, int>>& shapes, int leaf, NDPlan& plan,
              std::string& err);

}  // namespace hddm
