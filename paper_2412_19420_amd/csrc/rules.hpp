// Association rules over a mining result (k_rules.hip).
#pragma once

#include "internal.hpp"

namespace bm {

// Longest itemset whose rules can be listed: antecedents are bit masks over
// the itemset's positions, enumerated 2^L - 2 per itemset.
constexpr uint32_t RULE_MAX_LEN = 24;
constexpr uint32_t RULE_DEFAULT_LEN = 20;

// One result slice (nF itemsets in canonical order: offs[nF + 1] into items,
// supports supp) and the rule arrays of the emit pass.
struct RuleArgs {
  const uint64_t* offs;
  const uint32_t* items;
  const uint32_t* supp;
  uint64_t nF;
  uint64_t n;             // transactions of the database
  uint32_t min_conf_ppm;  // rule kept iff supp(Z) * 10^6 >= min_conf_ppm * supp(X)
  uint32_t max_len;       // itemsets longer than this give no rules
  uint32_t* count;        // count pass: rules per itemset
  const uint64_t* pos;    // emit pass: first rule of each itemset
  uint32_t* status;       // set to non-zero if a subset was missing from the list
  uint64_t* rz;
  uint32_t *rmask, *rsx, *rsy, *rsz;
  double *rconf, *rlift;
};

void launch_rules_count(const RuleArgs& a, hipStream_t s);
void launch_rules_emit(const RuleArgs& a, hipStream_t s);

}  // namespace bm
