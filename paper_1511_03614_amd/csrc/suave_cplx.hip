// Subregion-adaptive Monte Carlo, complex mode (nvmax up to 8): instances per variable class and
// internal order count.
#include "suave.hpp"

namespace sdi {

int launch_suave_cplx(int nvmax, int km, const SuaveArgs& a, hipStream_t st) {
  if (a.nreg <= 0) return 0;
  constexpr int WPB = BLOCK / 64;
  const int64_t blocks = (a.nreg + WPB - 1) / WPB;
  const dim3 g((unsigned)(blocks < (1 << 20) ? blocks : (1 << 20))), b(BLOCK);
#define SDI_C(NV, KM) k_suave<NV, KM, true><<<g, b, 0, st>>>(a)
  if (nvmax > 8) return (int)hipErrorInvalidValue;
  if (km == 4) {
    if (nvmax <= 4) SDI_C(4, 4);
    else SDI_C(8, 4);
  } else {
    if (nvmax <= 4) SDI_C(4, 8);
    else SDI_C(8, 8);
  }
#undef SDI_C
  return (int)hipGetLastError();
}

}  // namespace sdi
