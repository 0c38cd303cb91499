// Observables (internal interface).
#pragma once
#include "common.h"

namespace qrtebd {

constexpr int kMaxSites = 256;

struct EntropyArgs {
  const double* xi[kMaxSites];
  int chi[kMaxSites];
};

// Doubles of partial-sum workspace expect_run needs.
size_t expect_part_doubles(int chiL, int chiR);

// val (2 doubles) = sum conj(M) O M / |M|^2 and norm = |M|^2 over a tensor
// T[chiL][dd][chiR] with M = diag(xi) T (xi nullable); O is dd x dd.
int expect_run(const void* T, int prec, const double* xi, int chiL, int dd, int chiR, const c128* O, double* part,
               double* val, double* norm, hipStream_t s);

// out[m] = -sum p ln p with p = xi_m^2 / |xi_m|^2 for m < n.
int entropy_run(const EntropyArgs& a, int n, double* out, hipStream_t s);

}  // namespace qrtebd
