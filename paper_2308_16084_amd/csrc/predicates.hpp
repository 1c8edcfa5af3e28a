// Exact-sign geometric predicates on double coordinates.
//
// A floating-point evaluation is accepted when its magnitude exceeds a bound
// on its rounding error; otherwise the determinant is evaluated exactly with
// floating-point expansion arithmetic (Shewchuk, "Adaptive Precision
// Floating-Point Arithmetic and Fast Robust Geometric Predicates", 1997:
// two-sum, two-product, expansion sum and scaling, restated here).
#pragma once

namespace p2m {

// Sign of det[b-a, c-a, d-a]: +1 when d lies on the side of the plane (a,b,c)
// that the normal (b-a)x(c-a) points to.
int orient3d(const double* a, const double* b, const double* c, const double* d);

// For (a,b,c,d) with orient3d > 0: +1 when e lies strictly inside the sphere
// through a,b,c,d, -1 when strictly outside, 0 on it.
int insphere(const double* a, const double* b, const double* c, const double* d, const double* e);

// Counters of how often the exact paths ran (statistics only).
long long predicate_exact_calls();

}  // namespace p2m
