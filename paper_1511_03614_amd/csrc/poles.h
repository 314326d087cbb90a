// Reduction of sectors with a_j < -1 (poles_host.cpp).
#pragma once
#include <complex>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sdint.h"

namespace sdi {

constexpr int POLE_SERIES_LEN = 12;   // coefficient series terms kept

// Arrays a reduced sector's descriptor points into.
struct PoleStore {
  std::vector<double> a, b, gam, del, coef;
  std::vector<int32_t> nterms;
  std::vector<uint8_t> exps;
};

// The problem's sectors with every a_j >= -1: input sectors without a_j < -1
// as given (series 1), the others replaced by their parts; descs point into
// the caller's arrays or into store.
struct PoleExpansion {
  std::vector<sdi_sector_desc> descs;
  std::vector<std::vector<std::complex<double>>> series;   // coefficient series per part
  std::vector<int> origin;                                  // input sector of each part
  std::vector<std::shared_ptr<PoleStore>> store;
};

int expand_poles(const sdi_problem_desc* d, PoleExpansion& out, std::string& err);

}  // namespace sdi
