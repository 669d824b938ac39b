"""Address map and checksum sinks of the K-load sweep (oracle side).

What the method computes (Section 3, "Instruments" and "The axis K"): every
thread issues K independent loads per iteration, and every loaded word is
folded into a sink.  The sweep keeps two sinks per lane, a wrapping 32-bit
sum and a 32-bit XOR, and reduces them over the lanes of a wave and over
the grid with the same two operators.  Both operators are associative and
commutative, so the result depends only on WHICH words each lane loads.

Address map (Section 3, "Fixed-work control": whatever K is, a wave's loads
stay one contiguous, coalesced run; K only sets how many loads each lane has
outstanding):

    work unit     wave-group q = 0 .. Q-1, dealt to the waves round robin
                  (wave w of n_waves handles q = w, w + n_waves, ...) or in
                  blocks (wave w handles a contiguous range of groups); see
                  ``plan.groups_of_wave``
    load j of K   lane l reads vector  v = ((q*K + j)*64 + l) mod n_vec
                  of a region of n_vec vectors of V bytes, starting at
                  vector ``base`` of the buffer; in the strided layout
                  (the address-ordering experiment Section 4.2 proposes)
                  v = ((j*Q + q)*64 + l) mod n_vec instead.

A vector of V bytes is V/4 consecutive little-endian 32-bit words.

All sums are kept in uint64 NumPy arrays (wrapping modulo 2**64, which is
consistent modulo 2**32) and reduced to uint32 at the end.
"""
import numpy as np

from . import plan, splitmix

WAVE = 64
MASK32 = np.uint64(0xFFFFFFFF)


def vector_index(q, j, lane, K, n_vec, Q=None, order=plan.ROUND_ROBIN):
    """Vector read by ``lane`` for load ``j`` of wave-group ``q``: the K
    loads of a group are adjacent 64-lane segments, (q*K + j)*64 + lane;
    in the strided layout they are Q segments apart, (j*Q + q)*64 + lane."""
    if order == plan.STRIDED:
        return ((j * Q + q) * WAVE + lane) % n_vec
    return ((q * K + j) * WAVE + lane) % n_vec


def _group_vectors(q0, q1, K, n_vec, Q=None, order=plan.ROUND_ROBIN):
    """Vector indices of groups q0..q1-1 as an array [groups, K, 64]."""
    if order == plan.STRIDED:
        q = np.arange(q0, q1, dtype=np.int64)[:, None, None]
        j = np.arange(K, dtype=np.int64)[None, :, None]
        lane = np.arange(WAVE, dtype=np.int64)[None, None, :]
        return ((j * Q + q) * WAVE + lane) % n_vec
    f = np.arange(q0 * K * WAVE, q1 * K * WAVE, dtype=np.int64)
    return (f % n_vec).reshape(q1 - q0, K, WAVE)


def _region(words_u32, V, base, n_vec):
    """View the region as [n_vec, V/4] words."""
    wpv = V // 4
    flat = words_u32[base * wpv:(base + n_vec) * wpv]
    if flat.size != n_vec * wpv:
        raise ValueError("region exceeds the buffer")
    return flat.reshape(n_vec, wpv)


def per_lane(words_u32, V, K, Q, n_waves, base=0, n_vec=None,
             chunk_groups=4096, order=plan.ROUND_ROBIN):
    """Per-lane (sum32, xor32), each a uint32 array [n_waves, 64]."""
    if n_vec is None:
        n_vec = words_u32.size * 4 // V - base
    vec = _region(words_u32, V, base, n_vec)
    s = np.zeros((n_waves, WAVE), dtype=np.uint64)
    x = np.zeros((n_waves, WAVE), dtype=np.uint32)
    for q0 in range(0, Q, chunk_groups):
        q1 = min(Q, q0 + chunk_groups)
        v = _group_vectors(q0, q1, K, n_vec, Q, order)    # [g, K, 64]
        w = vec[v]                                          # [g, K, 64, V/4]
        gs = w.astype(np.uint64).sum(axis=(1, 3))           # [g, 64]
        gx = np.bitwise_xor.reduce(w, axis=3)
        gx = np.bitwise_xor.reduce(gx, axis=1)              # [g, 64]
        owner = _owners(q0, q1, Q, n_waves, order)
        np.add.at(s, owner, gs)
        np.bitwise_xor.at(x, owner, gx)
    return (s & MASK32).astype(np.uint32), x


def _owners(q0, q1, Q, n_waves, order):
    q = np.arange(q0, q1)
    if order in (plan.ROUND_ROBIN, plan.STRIDED):
        return q % n_waves
    return q // -(-Q // n_waves)


def per_wave(words_u32, V, K, Q, n_waves, base=0, n_vec=None,
             chunk_groups=4096, order=plan.ROUND_ROBIN):
    """Per-wave (sum32, xor32), each a uint32 array [n_waves]."""
    if n_vec is None:
        n_vec = words_u32.size * 4 // V - base
    vec = _region(words_u32, V, base, n_vec)
    s = np.zeros(n_waves, dtype=np.uint64)
    x = np.zeros(n_waves, dtype=np.uint32)
    for q0 in range(0, Q, chunk_groups):
        q1 = min(Q, q0 + chunk_groups)
        v = _group_vectors(q0, q1, K, n_vec, Q, order)
        w = vec[v].reshape(q1 - q0, -1)                     # [g, K*64*V/4]
        gs = w.astype(np.uint64).sum(axis=1)
        gx = np.bitwise_xor.reduce(w, axis=1)
        owner = _owners(q0, q1, Q, n_waves, order)
        np.add.at(s, owner, gs)
        np.bitwise_xor.at(x, owner, gx)
    return (s & MASK32).astype(np.uint32), x


def combine(sums, xors):
    """Reduce partial (sum32, xor32) arrays to one pair of Python ints."""
    s = int(np.asarray(sums, dtype=np.uint64).sum() & MASK32)
    x = int(np.bitwise_xor.reduce(np.asarray(xors, dtype=np.uint32).ravel()))
    return s, x


def whole_buffer(words_u32):
    """(sum32, xor32) of every word of a buffer, each word once."""
    s = int(words_u32.astype(np.uint64).sum() & MASK32)
    x = int(np.bitwise_xor.reduce(words_u32)) if words_u32.size else 0
    return s, x


def wave_from_seed(seed, V, K, Q, n_waves, wave, base=0, n_vec=None,
                   buffer_bytes=None, order=plan.ROUND_ROBIN):
    """(sum32, xor32) of one wave, generating only the words it reads.

    Used for sampled checks on buffers too large to hold on the host: the
    generator is counter-based, so word i is computed from (seed, i) alone.
    Exactly one of ``n_vec`` / ``buffer_bytes`` gives the region size (the
    region defaults to the whole buffer).
    """
    if n_vec is None:
        n_vec = buffer_bytes // V - base
    wpv = V // 4
    s = 0
    x = 0
    for q in plan.groups_of_wave(wave, Q, n_waves, order):
        f = _group_vectors(q, q + 1, K, n_vec, Q, order).ravel() + base
        # runs of consecutive vectors (one per segment at most, or the whole
        # group when its loads are adjacent); generate run by run
        starts = np.flatnonzero(np.diff(f) != 1) + 1
        for run in np.split(f, starts):
            w = splitmix.words(seed, int(run[0]) * wpv, run.size * wpv)
            s += int(w.astype(np.uint64).sum())
            x ^= int(np.bitwise_xor.reduce(w))
    return s & 0xFFFFFFFF, x


def lane_from_seed(seed, V, K, Q, n_waves, wave, lane, n_vec,
                   order=plan.ROUND_ROBIN):
    """(sum32, xor32) of one lane, generating only the words it reads."""
    wpv = V // 4
    s = 0
    x = 0
    for q in plan.groups_of_wave(wave, Q, n_waves, order):
        for j in range(K):
            v = vector_index(q, j, lane, K, n_vec, Q, order)
            w = splitmix.words(seed, v * wpv, wpv)
            s += int(w.astype(np.uint64).sum())
            x ^= int(np.bitwise_xor.reduce(w))
    return s & 0xFFFFFFFF, x


def two_stream_regions(n_vec_total):
    """Vector regions of the two co-resident streams.

    Stream A (plain waves) reads vectors [0, M/2) and stream B (LDS-async
    waves) reads [M/2, M), with M the buffer's vector count; each stream
    has its own wave-group count and its own round-robin over its waves.
    """
    half = n_vec_total // 2
    return (0, half), (half, n_vec_total - half)


def range_sinks(seed, word_start, n_words, chunk=1 << 22):
    """Global (sum32, xor32) of the seeded buffer's words
    [word_start, word_start + n_words).

    A launch that reads a contiguous region exactly once (a pass with no
    wrap: Q wave-groups of K*64 consecutive vectors from the region's
    start) folds exactly these words, and both sinks are associative and
    commutative, so this is its global result whatever the dealing of
    groups to waves."""
    s = 0
    x = 0
    for a in range(word_start, word_start + n_words, chunk):
        w = splitmix.words(seed, a, min(chunk, word_start + n_words - a))
        s += int(w.astype(np.uint64).sum())
        x ^= int(np.bitwise_xor.reduce(w)) if w.size else 0
    return s & 0xFFFFFFFF, x


def range_sinks_many(ranges, threads=1, piece=1 << 24):
    """``range_sinks`` of many (seed, word_start, n_words) ranges, in
    pieces of at most ``piece`` words evaluated on ``threads`` threads
    (NumPy releases the interpreter lock inside its array loops); the
    pieces of a range are combined with the sinks' own operators.  Equal
    ranges are computed once."""
    from concurrent.futures import ThreadPoolExecutor
    uniq = sorted(set(ranges))
    tasks = []
    for k, (seed, start, n) in enumerate(uniq):
        for a in range(start, start + n, piece):
            tasks.append((k, seed, a, min(piece, start + n - a)))

    def run(t):
        return t[0], range_sinks(t[1], t[2], t[3])

    if threads > 1:
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(run, tasks))
    else:
        parts = [run(t) for t in tasks]
    acc = [[0, 0] for _ in uniq]
    for k, (s, x) in parts:
        acc[k][0] = (acc[k][0] + s) & 0xFFFFFFFF
        acc[k][1] ^= x
    got = {r: tuple(a) for r, a in zip(uniq, acc)}
    return [got[r] for r in ranges]
