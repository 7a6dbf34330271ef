"""CPU oracle for Boolean-matrix frequent-itemset mining.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute anything in this package; only the tests, the smoke entry point and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library.

What it computes (paper, Section III):
  * the transaction x item Boolean matrix M, M[i,j] = 1 iff item j is in
    transaction i (Eq. 1), with set semantics: duplicate ids in a row collapse;
  * the support of an itemset X, S(X) = number of rows i with M[i,j] = 1 for
    every j in X -- Eq. 2 for pairs, extended to longer sets by ANDing further
    columns one after another;
  * the frequent itemsets: every non-empty X with S(X) >= minsup, where minsup is
    an absolute count (the paper's strict S(X) > theta is minsup = floor(theta)+1;
    see `paper_theta_to_minsup`).

Output convention shared by every function here: a list of (itemset, support)
with each itemset an ascending tuple of item ids and the list in lexicographic
order of those tuples (a proper prefix precedes its extensions).

Modules:
  sets     plain Python-set miner (the reference definition, small inputs)
  brute    exhaustive enumeration of all 2^m - 1 itemsets (m <= 16)
  pairs    closed-form pair-support matrix A^T A (Eq. 2)
  certify  certificate checker for a claimed result at any size
  cpp      ctypes wrapper of oracle.cpp (sorted tid-vector miner, multi-threaded)
  mlp      float64 forward/backward of the scheduler's cost model
"""
