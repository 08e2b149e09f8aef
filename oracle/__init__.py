"""CPU oracle for sparse-tensor transposition (Quesadilla, Mueller et al., arXiv 2005.10427).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links or
executes anything in this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg may.  It shares no code with the HIP library: the
only thing both sides consume is the seeded input generator in ``datagen``.

Contents (each function cites the paper passage it restates):

* ``transpose``     -- the definition: a stable sort of the nonzeros under the
                       lexicographic order sigma (Sec. 2, Sec. 2.1), followed by
                       a bitwise gather of coordinates and values.
* ``brute``         -- the same result with no sort at all (dense enumeration of
                       the coordinate space in sigma order); pins ``transpose``.
* ``planner``       -- the follow-set f, the lower bound b, the output orders of
                       both PartialSort variants and QuesadillaSort (Alg. 3),
                       Top-K-sadilla's target order and the full LSD radix plan.
* ``partial_sort``  -- Alg. 1 and Alg. 2 executed step by step on a list of
                       coordinate tuples, and a plan executor built on them.
* ``csf``           -- compressed-sparse-fiber packing of a sigma-sorted COO
                       tensor and its expansion back to COO.
* ``mlp``           -- fp64 forward/backward/Adam of the schedule-selector MLP
                       (the true-cost model the paper proposes in Sec. 5).
* ``features``      -- the selector's 32 features: sampled counts per mode and
                       the pass/bit counts of the three schedules.
* ``invariants``    -- checks that hold for any correct transposition.

Parity status: every function above is pinned by tests that do not re-type its
formula (worked example of Sec. 3.3, brute-force enumeration, closed forms,
the pass-count figure of Sec. 4.2, finite differences for the MLP, published
SplitMix64 outputs, brute-force recounts of the feature counts).
"""
