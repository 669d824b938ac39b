"""Pointer chase (oracle side): the latency probe of Section 4.1 follows a
dependent chain idx <- chain[idx]; its only arithmetic result is the index
reached, which is the chain followed that many times."""


def follow(words, start, hops):
    """Index reached from ``start`` after ``hops`` dependent loads."""
    idx = int(start)
    for _ in range(int(hops)):
        idx = int(words[idx])
    return idx


def cycle_length(words, start, limit):
    """Hops until the chain first returns to ``start`` (None past limit)."""
    idx = int(words[start])
    n = 1
    while idx != start:
        if n >= limit:
            return None
        idx = int(words[idx])
        n += 1
    return n
