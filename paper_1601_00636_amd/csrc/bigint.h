// Exact CPU arithmetic for root confirmation (see bigint.cpp).
#pragma once

#include <stdint.h>

#include <string>

namespace cuboid {

// Q_pq(t) == 0 exactly; *ok is false if an intermediate overflowed.
bool exact_is_root(uint32_t p, uint32_t q, uint64_t t, bool *ok);
// Q_pq(t) as a signed decimal string.
bool exact_value_decimal(uint32_t p, uint32_t q, uint64_t t, std::string *out);
// Theorem 1.1 inequality bits: t > p^2, t > pq, t > q^2, (p^2 + t)(pq + t) > 2 t^2.
uint32_t theorem_flags(uint32_t p, uint32_t q, uint64_t t);

}  // namespace cuboid
