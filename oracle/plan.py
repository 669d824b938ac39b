"""Fixed-work control and exact-work accounting (oracle side).

Section 3 ("Fixed-work control") divides L, the target number of logical
loads, by threads x K to get a cell's iteration count, so that every K
issues about the same number of logical loads.  Section 4.2 ("Exact-work accounting")
judges the match on iterations times loads per thread, counted exactly,
and prints the largest mismatch over K in {1,2,4,8} as 0.024576 %.

Three ways of turning (L, K, grid) into work are written out here:

``per_thread_floor``  the paper's construction: every thread runs
                      floor(L / (threads * K)) iterations of K loads.
``wave_group``        the library's fixed-work mode: the work unit is a
                      wave-group (one wavefront's K coalesced 64-lane
                      loads), Q = floor(L / (64 K)) groups are dealt to the
                      waves round-robin, so iteration counts differ by at
                      most one between waves.  Its K-set mismatch over
                      K = 1..16 at L = 2**26 is below 1e-5.
``fixed_iters``       the paper's baseline arm (Table 1, first row): every
                      wave runs the same iteration count, so issued work
                      grows in proportion to K.

Mismatch over a K set is (max - min) / max of the issued counts; the
denominator is the set maximum (this reading reproduces 0.024576 %).
"""

WAVE = 64


def per_thread_floor(L, threads, K):
    """Paper's construction: iterations per thread and issued logical loads."""
    if threads <= 0 or K <= 0:
        raise ValueError("threads and K must be positive")
    iters = L // (threads * K)
    return {"iters": iters, "loads_per_thread": iters * K,
            "issued": iters * K * threads}


ROUND_ROBIN, BLOCKED, STRIDED = 0, 1, 2


def groups_of_wave(w, Q, n_waves, order=ROUND_ROBIN):
    """The wave-groups wave ``w`` handles, in the order it handles them.

    round robin: q = w, w + n_waves, ... (neighbouring waves read
                 neighbouring groups at the same time);
    blocked:     q = w*G .. w*G + G - 1 with G = ceil(Q / n_waves) (every
                 wave streams its own contiguous range);
    strided:     dealt as round robin (only the loads' addresses differ,
                 see ``checksums.vector_index``).
    Either way every group below Q is handled exactly once.
    """
    if order in (ROUND_ROBIN, STRIDED):
        return range(w, Q, n_waves)
    G = -(-Q // n_waves)
    return range(min(Q, w * G), min(Q, (w + 1) * G))


def owner(q, Q, n_waves, order=ROUND_ROBIN):
    """The wave that handles group ``q``."""
    if order in (ROUND_ROBIN, STRIDED):
        return q % n_waves
    return q // -(-Q // n_waves)


def wave_group(L, K, n_waves, order=ROUND_ROBIN):
    """Wave-group fixed-work plan: Q = floor(L / 64K) groups over n_waves."""
    if K <= 0 or n_waves <= 0:
        raise ValueError("K and n_waves must be positive")
    Q = L // (WAVE * K)
    iters = [len(groups_of_wave(w, Q, n_waves, order)) for w in range(n_waves)]
    return {"Q": Q, "issued": WAVE * K * Q, "iters": iters,
            "iters_min": min(iters), "iters_max": max(iters)}


def fixed_iters(iters, K, n_waves):
    """Baseline arm: every wave runs ``iters`` iterations of K loads."""
    Q = n_waves * iters
    return {"Q": Q, "issued": WAVE * K * Q, "iters": [iters] * n_waves,
            "iters_min": iters, "iters_max": iters}


def kset_mismatch(issued_counts):
    """(max - min) / max over the issued counts of a K set (a fraction)."""
    hi, lo = max(issued_counts), min(issued_counts)
    if hi == 0:
        raise ValueError("no work issued")
    return (hi - lo) / hi


def target_mismatch(L, issued):
    """Shortfall of one cell against its target: (L - issued) / L."""
    return (L - issued) / L
