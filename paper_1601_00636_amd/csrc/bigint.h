// Exact CPU arithmetic for root confirmation (see bigint.cpp).
#pragma once

#include <stdint.h>

#include <string>

namespace cuboid {

// t = t_hi 2^64 + t_lo throughout.
// Q_pq(t) == 0 exactly; *ok is false for t >= 2^70 (outside the width).
bool exact_is_root(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi, bool *ok);
// Q_pq(t) as a signed decimal string; false for t >= 2^70.
bool exact_value_decimal(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi, std::string *out);
// Theorem 1.1 inequality bits: t > p^2, t > pq, t > q^2, (p^2 + t)(pq + t) > 2 t^2.
uint32_t theorem_flags(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi);

}  // namespace cuboid
