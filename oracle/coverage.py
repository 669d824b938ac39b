"""Which cache lines a cell reads, and how often (oracle side).

Section 4.2 ("Allocation-size sweep") bounds the unique coverage of its
largest allocation by the issued volume over the allocation (16,785 MiB
over 20,000 MiB, at most 84 %) because it collects no address trace, and
the discriminating experiment proposed after Table 2 asks for
address-trace coverage.  The address map makes the trace exact: load j of
wave-group q covers the 64-lane segment (64 consecutive vectors) number
(q*K + j) mod n_seg of the allocation (or (j*Q + q) mod n_seg in the
strided layout), where n_seg = n_vec / 64, and every group below Q is
handled by exactly one wave (``plan.groups_of_wave``).

``segment_reads`` walks every wave's groups in the order that wave handles
them and counts the reads of every segment; ``line_coverage`` turns the
counts into 128-byte-line figures: unique lines touched over the
allocation's lines, total line reads and re-reads (reads beyond the first
of a line).  Order changes who reads a segment and when, never how often.

``lane_line_reads`` is a pure-Python brute force over every lane's vector
for tiny cells.
"""
import numpy as np

from . import plan

WAVE = 64
LINE = 128


def segment_reads(alloc_bytes, V, K, Q, n_waves, order=plan.ROUND_ROBIN):
    """Reads of every 64-lane segment (64*V bytes) of the allocation."""
    n_seg = alloc_bytes // V // WAVE
    if n_seg * WAVE * V != alloc_bytes:
        raise ValueError("allocation must be whole 64-lane segments")
    if order == plan.STRIDED:
        # load j of group q reads segment (j*Q + q) mod n_seg
        counts = np.zeros(n_seg, dtype=np.int64)
        for w in range(n_waves):
            g = plan.groups_of_wave(w, Q, n_waves, order)
            q = np.arange(g.start, g.stop, g.step, dtype=np.int64)
            for j in range(K):
                np.add.at(counts, (j * Q + q) % n_seg, 1)
        return counts
    diff = np.zeros(n_seg + 1, dtype=np.int64)
    for w in range(n_waves):
        g = plan.groups_of_wave(w, Q, n_waves, order)
        q = np.arange(g.start, g.stop, g.step, dtype=np.int64)
        if q.size == 0:
            continue
        first = (q * K) % n_seg
        # K consecutive segments from `first`, cut where they wrap
        end = first + K
        plain = end <= n_seg
        np.add.at(diff, first[plain], 1)
        np.add.at(diff, end[plain], -1)
        wr = ~plain
        if np.any(wr):
            np.add.at(diff, first[wr], 1)
            diff[n_seg] -= int(wr.sum())
            # the wrapped part [0, end - n_seg), possibly several passes if
            # K exceeds the segment count
            rest = end[wr] - n_seg
            full, part = np.divmod(rest, n_seg)
            diff[0] += int(full.sum())
            diff[n_seg] -= int(full.sum())
            np.add.at(diff, np.zeros(part.size, dtype=np.int64), 1)
            np.add.at(diff, part, -1)
    return np.cumsum(diff)[:n_seg]


def line_coverage(alloc_bytes, V, K, Q, n_waves, order=plan.ROUND_ROBIN):
    """Unique 128-byte lines touched, the allocation's lines, total line
    reads, re-reads and the most reads of one line, for a whole cell."""
    seg = segment_reads(alloc_bytes, V, K, Q, n_waves, order)
    lps = WAVE * V // LINE                      # lines per segment (V/2)
    unique = int(np.count_nonzero(seg)) * lps
    total = int(seg.sum()) * lps
    return {"unique_lines": unique, "alloc_lines": alloc_bytes // LINE,
            "line_reads": total, "re_reads": total - unique,
            "max_reads": int(seg.max()) if seg.size else 0,
            "coverage": unique / (alloc_bytes // LINE)}


def lane_line_reads(alloc_bytes, V, K, Q, n_waves, order=plan.ROUND_ROBIN):
    """Brute force: per-line read counts from every lane's vector.  A
    64-lane load reads each line it touches once, so a line counts once per
    (group, load) that touches it."""
    n_vec = alloc_bytes // V
    counts = [0] * (alloc_bytes // LINE)
    for w in range(n_waves):
        for q in plan.groups_of_wave(w, Q, n_waves, order):
            for j in range(K):
                lines = set()
                seg = j * Q + q if order == plan.STRIDED else q * K + j
                for lane in range(WAVE):
                    v = (seg * WAVE + lane) % n_vec
                    lines.add(v * V // LINE)
                for ln in lines:
                    counts[ln] += 1
    return counts
