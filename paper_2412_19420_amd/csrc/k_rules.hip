// Association rules from the mined frequent itemsets: for each frequent Z and
// each split Z = X + Y into non-empty disjoint parts, confidence
// supp(Z) / supp(X) and lift supp(Z) n / (supp(X) supp(Y)).  The paper names
// association rule learning as the use of frequent itemsets (abstract,
// Section I) and support, confidence and lift as its indicators (Section IV-A).
//
// Every subset of a frequent set is frequent, so supp(X) and supp(Y) are
// looked up in the mined list itself: a join of the list with itself.  The
// list is in canonical order (ascending tuples, lexicographic, a prefix before
// its extensions), so each lookup is a binary search of tuple comparisons.
//
// One wave per itemset Z of L items.  The antecedents X are the non-empty
// subsets of Z's positions in preorder of the subset trie -- exactly the
// lexicographic order of X as a tuple -- so lanes take consecutive ranks, turn
// each rank into a subset mask, look up both sides and test the threshold in
// integers: supp(Z) * 10^6 >= min_conf_ppm * supp(X).  A count pass gives
// each Z's number of rules; after a scan, the emit pass places every rule by
// the ballot ranks of its 64-rank chunk, so the output comes out in order
// (Z's position, then X) with no sort.
#include "internal.hpp"
#include "rules.hpp"

namespace bm {

namespace {

constexpr int kWaves = 4;  // waves per workgroup
constexpr uint32_t kRuleOk = 0, kRuleMissing = 1;

// Orders one wave's LDS writes before its own later reads (and reads before
// later writes): a wave's LDS operations are performed in issue order, and the
// fence keeps the compiler from moving them across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Non-empty subsets of L positions in preorder of the subset trie: the sets
// whose smallest position is p form one subtree of 2^(L-1-p) sets, and inside
// it {p} comes first, followed by the subtrees of the positions after p.
__device__ inline uint32_t unrank_subset(uint32_t r, uint32_t L) {
  uint32_t mask = 0, p = 0;
  for (;;) {
    const uint32_t size = 1u << (L - 1 - p);
    if (r < size) {
      mask |= 1u << p;
      if (r == 0) break;
      r -= 1;
    } else {
      r -= size;
    }
    ++p;
  }
  return mask;
}

// Position in [0, nF) of the itemset made of the items of z (LDS) selected by
// mask, or nF when it is missing.  Tuples compare item by item; a proper
// prefix comes first.
__device__ inline uint64_t find_set(const uint32_t* __restrict__ z, uint32_t mask,
                                    const uint64_t* __restrict__ offs,
                                    const uint32_t* __restrict__ items, uint64_t nF) {
  const uint32_t k = __popc(mask);
  uint64_t lo = 0, hi = nF;  // search [lo, hi)
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    const uint64_t a = offs[mid], len = offs[mid + 1] - a;
    int c = 0;  // sign of (X - F[mid])
    uint32_t m = mask;
    for (uint64_t t = 0;; ++t) {
      if (t == k || t == len) {
        c = (t == k && t == len) ? 0 : (t == k ? -1 : 1);
        break;
      }
      const uint32_t x = z[__ffs(m) - 1];
      m &= m - 1;
      const uint32_t f = items[a + t];
      if (x != f) {
        c = x < f ? -1 : 1;
        break;
      }
    }
    if (c == 0) return mid;
    if (c < 0) hi = mid; else lo = mid + 1;
  }
  return nF;
}

template <bool EMIT>
__global__ __launch_bounds__(64 * kWaves) void k_rules(RuleArgs a) {
  __shared__ uint32_t s_z[kWaves][RULE_MAX_LEN];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* z = s_z[wv];
  const uint64_t nwaves = (uint64_t)gridDim.x * kWaves;
  for (uint64_t zi = (uint64_t)blockIdx.x * kWaves + wv; zi < a.nF; zi += nwaves) {
    const uint64_t a0 = a.offs[zi];
    const uint32_t L = (uint32_t)(a.offs[zi + 1] - a0);
    if (L < 2 || L > a.max_len) {
      if (!EMIT && lane == 0) a.count[zi] = 0;
      continue;
    }
    if (lane < (int)L) z[lane] = a.items[a0 + lane];
    wave_lds_sync();
    const uint64_t sz = a.supp[zi];
    const uint32_t full = (1u << L) - 1;
    const uint32_t total = full;  // ranks of the non-empty subsets
    uint64_t out = EMIT ? a.pos[zi] : 0;
    uint32_t cnt = 0;
    for (uint32_t base = 0; base < total; base += 64) {
      const uint32_t r = base + (uint32_t)lane;
      bool pass = false;
      uint32_t mask = 0, sx = 0, sy = 0;
      if (r < total) {
        mask = unrank_subset(r, L);
        if (mask != full) {
          const uint64_t ix = find_set(z, mask, a.offs, a.items, a.nF);
          const uint64_t iy = find_set(z, full & ~mask, a.offs, a.items, a.nF);
          if (ix == a.nF || iy == a.nF) {
            atomicOr(a.status, kRuleMissing);
          } else {
            sx = a.supp[ix];
            sy = a.supp[iy];
            pass = sz * 1000000ull >= (uint64_t)a.min_conf_ppm * sx;
          }
        }
      }
      const uint64_t bal = __ballot(pass);
      if (EMIT && pass) {
        const uint64_t o = out + (uint64_t)__popcll(bal & ((1ull << lane) - 1));
        a.rz[o] = zi;
        a.rmask[o] = mask;
        a.rsx[o] = sx;
        a.rsy[o] = sy;
        a.rsz[o] = (uint32_t)sz;
        a.rconf[o] = (double)sz / (double)sx;
        a.rlift[o] = (double)(sz * a.n) / (double)((uint64_t)sx * sy);
      }
      out += (uint64_t)__popcll(bal);
      cnt += (uint32_t)__popcll(bal);
    }
    if (!EMIT && lane == 0) a.count[zi] = cnt;
    wave_lds_sync();  // z is rewritten for the next itemset
  }
}

uint32_t rules_grid(uint64_t nF) {
  uint64_t g = (nF + kWaves - 1) / kWaves;
  if (g < 1) g = 1;
  const uint64_t cap = (uint64_t)cu_count() * 16;
  return (uint32_t)(g < cap ? g : cap);
}

}  // namespace

void launch_rules_count(const RuleArgs& a, hipStream_t s) {
  if (a.nF == 0) return;
  k_rules<false><<<rules_grid(a.nF), 64 * kWaves, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

void launch_rules_emit(const RuleArgs& a, hipStream_t s) {
  if (a.nF == 0) return;
  k_rules<true><<<rules_grid(a.nF), 64 * kWaves, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
