// Expression tapes: integrands given as text in the integration workers' input
// format (x[i], f[i], p[base,exponent], l[arg], P, G, + - * / and brackets),
// compiled on the host into straight-line code over numbered slots.  Shared by
// the host compiler and the HIP kernels (plain C++).
//
// Slots 0 .. n-1 hold the point's coordinates x[1] .. x[n]; every instruction
// writes one slot from up to two operands, each a slot or the instruction's
// constant, reading its operands before it writes.  The host allocates the
// remaining slots by liveness, so a slot is rewritten once its value is dead
// (an instruction may write the slot of an operand it reads for the last
// time).  The tape is padded with X_NOP to a multiple of EXPR_FETCH
// instructions, the number the device fetches per round of scalar loads.
//
// A complex tape (an integrand that uses the imaginary unit I) holds a
// complex value per slot: slot s is the pair of rows 2s (real part) and 2s + 1
// (imaginary part); constants in imm are real, X_IUNIT makes i.  The
// operations are complex: l[a] is the principal logarithm with arg = -pi on
// the negative real axis (the side an F - i0 prescription approaches), a^b for
// a non-integer b is exp(b l[a]), a^k for an integer k is taken by products.
#pragma once
#include <stdint.h>

namespace sdi {

enum ExprOp : uint8_t {
  X_CONST = 0,   // dst = imm
  X_ADD,         // dst = a + b
  X_SUB,         // dst = a - b
  X_MUL,         // dst = a * b
  X_DIV,         // dst = a / b
  X_NEG,         // dst = -a
  X_LOG,         // dst = ln a (NaN for a < 0)
  X_POWI,        // dst = a^k for the integer k (products, then one reciprocal if k < 0)
  X_POW,         // dst = a^b, C pow semantics (NaN for a < 0 and non-integer b)
  X_NOP,         // nothing (padding)
  X_IUNIT,       // dst = i (complex tapes)
};

constexpr uint8_t X_OPMASK = 0x1f;
constexpr uint8_t X_IMMA = 0x20;     // operand a is the constant imm
constexpr uint8_t X_IMMB = 0x40;     // operand b is the constant imm
constexpr int EXPR_FETCH = 8;

struct alignas(16) ExprIns {
  uint8_t op, dst, a, b;
  int32_t k;
  double imm;
};

constexpr int EXPR_MAX_SLOTS = 96;   // slots per point (LDS: 512 B each per wave)
constexpr int EXPR_MAX_SLOTS_CPLX = 48;   // complex slots per point (1 KiB each per wave)
constexpr int EXPR_BLOCK = 64;       // threads per block of the expression kernels (one wave)

struct ExprArgs {
  const ExprIns* ins;
  int32_t nins;
  int32_t nslots;
  int32_t out;                       // slot holding the integrand value
  int32_t cplx;                      // 1: complex tape
};

}  // namespace sdi
