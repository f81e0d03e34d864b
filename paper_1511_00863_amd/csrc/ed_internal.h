// Internal helpers shared by the host and device translation units of the library.
#pragma once
#include <cstdint>

namespace ed {

// Record an error text for ed_last_error() on this thread and return `code`.
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// Binomial coefficient C(n, k) for 0 <= n <= 64 (0 outside the triangle).
uint64_t binom(int n, int k);

// Lowest eigenvalue of a symmetric tridiagonal matrix by Sturm bisection.
double tridiag_lowest(const double *a, const double *b, int m);

}  // namespace ed
