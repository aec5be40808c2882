// Group sums of the BSGS plaintext-matrix product on the slots (App. A.4).
#pragma once
#include <cstddef>
#include <cstdint>

#include "internal.h"

namespace pfx {

// Terms of one launch: out = sum_t phi_g(pt[t]) (.) ct[t] (two polynomials).
constexpr int kMacTerms = 64;
struct MacTerms {
    const double *pt[kMacTerms];   // plaintext t, NTT domain, limb i at pt[t] + i N
    const double *ct[kMacTerms];   // degree-1 ciphertext t, limb i of poly p at ct[t] + p cs[t] + i N
    size_t cs[kMacTerms];
};

// out (poly stride so) = [out +] sum_{t < n_terms} phi_g(pt[t]) (.) ct[t] over
// nl limbs, canonical residues; g = 1 leaves the plaintexts as they are.
void launch_diag_mac(const Launch &L, double *out, size_t so, const MacTerms &m, int n_terms, int nl, uint32_t g,
                     bool accumulate);

}  // namespace pfx
