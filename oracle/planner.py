"""Oracle: the pass planner of Sec. 3.4-3.6, in the paper's notation.  TEST INFRASTRUCTURE ONLY.

Orders are tuples of modes.  Inside this module modes are 1-based, as in the
paper; the public helpers at the bottom take and return 0-based modes.

* follow(tau, p)            f(tau, p): the modes after p in tau (Sec. 3.4.1).
* lower_bound(tau, sigma)   b(tau, sigma): how many sigma_i have
                            f(sigma, sigma_i) not contained in f(tau, sigma_i)
                            (consequence of Lemma 3.2).
* partial_sort_order        output order of PartialSort(A, (tau_1..tau_l), tau_k):
                            tau_k moves to position l+1, the rest keep their
                            relative order (output equations of Alg. 1 / Alg. 2).
* quesadilla(sigma)         Alg. 3 for a simply ordered input.
* plan(tau_in, sigma)       Alg. 3 for any complete input order: the paper assumes
                            the simple input order without loss of generality
                            (Sec. 2.2), so the modes are relabelled by their
                            position in tau_in, planned, and mapped back.
* topk_target, topk_plan    Top-K-sadilla (Sec. 3.6): Quesadilla towards the
                            first K modes of sigma, then a complete sort of every
                            bucket of equal (sigma_1..sigma_K).
* lsd_plan                  full LSD radix sort: one histogram sort per mode,
                            least significant (sigma_r) first (Sec. 3).
"""


def follow(tau, p):
    """f(tau, p) = {tau_{k+1}, ..., tau_r} where tau_k = p."""
    tau = tuple(tau)
    k = tau.index(p)
    return frozenset(tau[k + 1:])


def lower_bound(tau, sigma):
    """b(tau, sigma): number of modes that every plan must sort on (Lemma 3.2)."""
    return sum(1 for m in sigma if not follow(sigma, m) <= follow(tau, m))


def partial_sort_order(tau, prefix_len, mode):
    """Order after PartialSort(A, (tau_1..tau_l), mode), for an A sorted under tau.

    Requires mode = tau_k with k > l.  Result: (tau_1..tau_l, tau_k,
    tau_{l+1}..tau_{k-1}, tau_{k+1}..tau_r); with l = 0 this is the
    non-bucketed output order.
    """
    tau = tuple(tau)
    k = tau.index(mode)  # 0-based position of tau_k
    if not k >= prefix_len:
        raise ValueError("PartialSort needs the sorted mode after the kept prefix")
    return tau[:prefix_len] + (mode,) + tau[prefix_len:k] + tau[k + 1:]


def quesadilla(sigma):
    """Alg. 3 (QuesadillaSort) for an input in the simple order (1, ..., r).

    sigma: complete order over modes 1..r.  Returns the list of calls
    PartialSort(A, prefix, mode) as (prefix tuple, mode), in execution order.
    """
    sigma = tuple(sigma)
    r = len(sigma)
    simple = tuple(range(1, r + 1))

    def s(i):  # sigma_i, 1-based
        return sigma[i - 1]

    calls = []
    l = 0
    while l < r:
        k = l
        # scan: extend while sigma_{k+1} still has to move (its follow set in
        # sigma is not already a subset of its follow set in the input order)
        while k + 1 < r and not follow(sigma, s(k + 1)) <= follow(simple, s(k + 1)):
            k += 1
        l_next = k + 1
        # sort: sigma_k, sigma_{k-1}, ..., sigma_{l+1}, each keeping the prefix
        # (sigma_1..sigma_l) already in place
        while k > l:
            calls.append((tuple(sigma[:l]), s(k)))
            k -= 1
        l = l_next
    return calls


def _to_positions(tau_in, sigma0):
    """Relabel 0-based modes as 1-based positions in the input order tau_in."""
    where = {m: i + 1 for i, m in enumerate(tau_in)}
    return tuple(where[m] for m in sigma0)


def _check(order, r):
    order = tuple(int(m) for m in order)
    if sorted(order) != list(range(r)):
        raise ValueError(f"{order} is not a complete order of {r} modes")
    return order


def plan(tau_in, sigma):
    """Minimal pass list for an input sorted under tau_in (0-based modes).

    Returns [(prefix modes, mode), ...]; an empty prefix means Alg. 1,
    otherwise Alg. 2 keeping that prefix.
    """
    r = len(sigma)
    tau_in = _check(tau_in, r)
    sigma = _check(sigma, r)
    calls = quesadilla(_to_positions(tau_in, sigma))
    back = lambda p: tau_in[p - 1]
    return [(tuple(back(p) for p in pre), back(m)) for pre, m in calls]


def apply_plan_orders(tau_in, calls):
    """Symbolic orders after each call, starting from tau_in (0-based modes)."""
    tau = tuple(tau_in)
    seen = [tau]
    for pre, m in calls:
        if tau[:len(pre)] != tuple(pre):
            raise ValueError(f"prefix {pre} is not in place in order {tau}")
        tau = partial_sort_order(tau, len(pre), m)
        seen.append(tau)
    return seen


def topk_target(tau_in, sigma, K):
    """Top-K-sadilla's intermediate order: (sigma_1..sigma_K) followed by the
    remaining modes in the order they have in tau_in (the Quesadilla target of
    Sec. 3.6 made complete)."""
    head = tuple(sigma[:K])
    rest = tuple(m for m in tau_in if m not in head)
    return head + rest


def topk_plan(tau_in, sigma, K):
    """(Quesadilla calls towards the Top-K target, K): the buckets of equal
    (sigma_1..sigma_K) are then each sorted completely to sigma order."""
    return plan(tau_in, topk_target(tau_in, sigma, K)), K


def lsd_plan(sigma):
    """Full LSD radix sort: Alg. 1 on sigma_r, then sigma_{r-1}, ..., sigma_1."""
    return [((), m) for m in reversed(tuple(sigma))]


def rl_minima(tau_in, sigma):
    """Modes sigma_i whose input position is below that of every later sigma_j.
    For a simply ordered input these are exactly the modes with
    f(sigma, sigma_i) contained in f(tau_in, sigma_i)."""
    pos = {m: i for i, m in enumerate(tau_in)}
    out = []
    for i, m in enumerate(sigma):
        if all(pos[m] < pos[x] for x in sigma[i + 1:]):
            out.append(m)
    return out
