// Checked int64 arithmetic of the public expression bytecode on the host
// (C semantics: truncating '/', '%' with the dividend's sign, arithmetic
// '>>', comparisons and logical operators give 0 or 1).  An operation that
// overflows, divides by zero or shifts by a count outside [0, 63] sets an
// error bit and yields 0, and evaluation goes on.
#pragma once
#include <stdint.h>
#include <algorithm>
#include "../../include/hgrd.h"
#include "hgrd_internal.h"

namespace hgrd {

inline int64_t hop(uint16_t op, int64_t a, int64_t b, uint32_t& err) {
  int64_t r;
  switch (op) {
    case RD_OP_ADD:
      if (__builtin_add_overflow(a, b, &r)) { err |= ERR_RANGE; return 0; }
      return r;
    case RD_OP_SUB:
      if (__builtin_sub_overflow(a, b, &r)) { err |= ERR_RANGE; return 0; }
      return r;
    case RD_OP_MUL:
      if (__builtin_mul_overflow(a, b, &r)) { err |= ERR_RANGE; return 0; }
      return r;
    case RD_OP_DIV:
    case RD_OP_MOD:
      if (b == 0) { err |= ERR_DIVZERO; return 0; }
      if (a == INT64_MIN && b == -1) { err |= ERR_RANGE; return 0; }
      return op == RD_OP_DIV ? a / b : a % b;
    case RD_OP_SHL: {
      if (b < 0 || b > 63) { err |= ERR_RANGE; return 0; }
      int64_t s = (int64_t)((uint64_t)a << b);
      if ((s >> b) != a) { err |= ERR_RANGE; return 0; }
      return s;
    }
    case RD_OP_SHR:
      if (b < 0 || b > 63) { err |= ERR_RANGE; return 0; }
      return a >> b;
    case RD_OP_AND: return a & b;
    case RD_OP_OR: return a | b;
    case RD_OP_XOR: return a ^ b;
    case RD_OP_MIN: return std::min(a, b);
    case RD_OP_MAX: return std::max(a, b);
    case RD_OP_LT: return a < b;
    case RD_OP_LE: return a <= b;
    case RD_OP_EQ: return a == b;
    case RD_OP_NE: return a != b;
    case RD_OP_GE: return a >= b;
    case RD_OP_GT: return a > b;
    case RD_OP_LAND: return (a != 0) && (b != 0);
    case RD_OP_LOR: return (a != 0) || (b != 0);
  }
  err |= ERR_INVAL;
  return 0;
}


}  // namespace hgrd
