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
  std::vector<int32_t> dmono;
};

// The problem's sectors with every a_j >= -1: input sectors without a_j < -1
// as given (series 1), the others replaced by their parts; descs point into
// the caller's arrays or into store.
struct PoleExpansion {
  std::vector<sdi_sector_desc> descs;
  std::vector<std::vector<std::complex<double>>> series;   // coefficient series per part
  std::vector<int> origin;                                  // input sector of each part
  std::vector<std::shared_ptr<PoleStore>> store;
  // set by separate_terms (empty otherwise): per part, the eps power its
  // integral is multiplied by is eps^-shift, and sub_only marks a part whose
  // subtraction keeps only the subtracted integrand (no boundary terms)
  std::vector<int> shift, sub_only;
};

int expand_poles(const sdi_problem_desc* d, PoleExpansion& out, std::string& err);
int separate_terms(PoleExpansion& X, std::string& err);

}  // namespace sdi
