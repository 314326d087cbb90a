// Integrator 4 (real mode): the partition phase (k_suave with DIV) and the
// final lattice phase, instances per variable class and internal order count.
#include "divonne.hpp"

namespace sdi {

template <class Args, class Launch>
static int by_class(int nvmax, int km, const Args& a, Launch&& L) {
  if (a.nreg <= 0) return 0;
  constexpr int WPB = BLOCK / 64;
  const int64_t blocks = (a.nreg + WPB - 1) / WPB;
  const dim3 g((unsigned)(blocks < (1 << 20) ? blocks : (1 << 20))), b(BLOCK);
  L(nvmax, km, g, b);
  return (int)hipGetLastError();
}

#define SDI_CLASSES(KERN)                     \
  if (km == 4) {                              \
    if (nvmax <= 4) KERN(4, 4);               \
    else if (nvmax <= 6) KERN(6, 4);          \
    else if (nvmax <= 8) KERN(8, 4);          \
    else if (nvmax <= 10) KERN(10, 4);        \
    else KERN(16, 4);                         \
  } else {                                    \
    if (nvmax <= 4) KERN(4, 8);               \
    else if (nvmax <= 6) KERN(6, 8);          \
    else if (nvmax <= 8) KERN(8, 8);          \
    else if (nvmax <= 10) KERN(10, 8);        \
    else KERN(16, 8);                         \
  }

int launch_divonne_part_real(int nvmax, int km, const SuaveArgs& a, hipStream_t st) {
  return by_class(nvmax, km, a, [&](int nvmax, int km, dim3 g, dim3 b) {
#define SDI_P(NV, KM) k_suave<NV, KM, false, true><<<g, b, 0, st>>>(a)
    SDI_CLASSES(SDI_P)
#undef SDI_P
  });
}

int launch_divonne_lattice_real(int nvmax, int km, const DivLatArgs& a, hipStream_t st) {
  return by_class(nvmax, km, a, [&](int nvmax, int km, dim3 g, dim3 b) {
#define SDI_L(NV, KM) k_divonne_lattice<NV, KM, false><<<g, b, 0, st>>>(a)
    SDI_CLASSES(SDI_L)
#undef SDI_L
  });
}

}  // namespace sdi
