"""Statistics of a K sweep.

Section 3 ("Timing, residency, statistics") and Section 4.2 fix the
reporting rules this module implements:

* one kernel launch is one sample; a cell's figure is the median over its
  launches, and the best launch is kept as a separate raw field
  (Section 4.1 reports median and best-of-N side by side);
* the post-peak change is (B(K=8) - B(K=2)) / B(K=2) on per-K medians
  (Section 4.2, Table 1), and per-launch paired changes are reported too
  (Section 4.2, "Repeatability");
* peak K and the knee follow a 95 % plateau rule whose last three cells
  must stay on the plateau (Section 3; Section 4.2, "Prevalence").  The paper does not spell
  the rule out; the reading used here: B* is the largest median, peak K
  the smallest K attaining it, knee the smallest K with B >= 0.95 B*;
  a curve is "saturating" if its last three cells are all >= 0.95 B*,
  else "rising-censored" if the peak is among the last three cells, else
  "peak-decline";
* a residency screen flags HBM-targeted cells whose attained bandwidth
  exceeds the HBM datasheet figure (Section 3);
* anomalous launches are disclosed rather than dropped (Section 4.2 and
  Limitations report two slow primary launches and keep medians).  The
  paper gives no threshold; the reading used here: a launch more than 10 %
  below its cell's median.

Little's law (Section 1, Section 2): offered bytes in flight equal
bandwidth times latency, so in-flight bytes / bandwidth is the implied
round-trip latency.
"""
import statistics

HBM_PEAK_GBPS = 8000.0            # MI355X HBM3E datasheet bandwidth
INFINITY_CACHE_BYTES = 256 << 20  # MI355X last-level (MALL) cache


def median(values):
    """Median of a non-empty sequence."""
    return statistics.median(list(values))


def decline(b2, b8):
    """(B8 - B2) / B2 as a fraction (negative for a decline)."""
    if b2 <= 0:
        raise ValueError("B(K=2) must be positive")
    return (b8 - b2) / b2


def per_k_medians(samples):
    """{K: [GB/s per launch]} -> {K: median}."""
    return {k: median(v) for k, v in samples.items() if len(v)}


def paired_declines(samples, k_lo=2, k_hi=8):
    """Per-launch changes B8[i]/B2[i] - 1 for launches present at both K."""
    a, b = samples[k_lo], samples[k_hi]
    return [decline(x, y) for x, y in zip(a, b)]


def peak_k(medians):
    """Smallest K whose median equals the largest median."""
    best = max(medians.values())
    return min(k for k, v in medians.items() if v == best)


def knee(medians, frac=0.95):
    """Smallest K whose median reaches frac * max median."""
    best = max(medians.values())
    return min(k for k, v in medians.items() if v >= frac * best)


def classify(medians, frac=0.95, tail=3):
    """Regime of a response curve: saturating / rising-censored / peak-decline."""
    ks = sorted(medians)
    if len(ks) < tail:
        raise ValueError("curve shorter than the stable tail")
    best = max(medians.values())
    last = ks[-tail:]
    if all(medians[k] >= frac * best for k in last):
        return "saturating"
    if peak_k(medians) in last:
        return "rising-censored"
    return "peak-decline"


def residency_flag(gbps, cell_bytes, datasheet_gbps=HBM_PEAK_GBPS,
                   cache_bytes=INFINITY_CACHE_BYTES):
    """True if an HBM-targeted cell reports more than the datasheet allows.

    Cells whose buffer fits in the last-level cache are not HBM-targeted and
    are never flagged (they may legitimately exceed the HBM figure).
    """
    return cell_bytes > cache_bytes and gbps > datasheet_gbps


def kset_mismatch(issued):
    """(max - min) / max over a K set's issued logical loads."""
    hi, lo = max(issued), min(issued)
    return (hi - lo) / hi


def in_flight_bytes(n_waves, K, vec_bytes, lanes=64):
    """Offered bytes in flight: every lane of every resident wave has K loads."""
    return n_waves * lanes * K * vec_bytes


def implied_latency_ns(in_flight, gbps):
    """Little's law: latency = bytes in flight / bandwidth (GB/s = bytes/ns)."""
    return in_flight / gbps


def anomalous_launches(samples, frac=0.9):
    """Launches below frac x their cell's median: [(K, GB/s, ratio)]."""
    out = []
    for k, v in sorted(samples.items()):
        if not v:
            continue
        m = median(v)
        out += [(k, x, x / m) for x in v if m > 0 and x < frac * m]
    return out


def front_duplicates(order, K, n_waves, Q, n_vec, max_iters=64):
    """Share of the loads of one lock-step iteration that read a 64-vector
    segment another load of the same iteration reads.

    Model of the f3 ordering experiment: every wave runs its i-th iteration
    at the same time, and the front is the K loads of every wave.  The
    owners: round robin (order 0) and strided (order 2) give wave w group
    q = i * n_waves + w, blocked (order 1) q = w * G + i (G = ceil(Q /
    n_waves)).  The segments: in the adjacent layouts (orders 0 and 1) load
    j of group q reads segment (q * K + j) mod S, in the strided one
    (j * Q + q) mod S, with S = n_vec / 64 segments in the allocation.
    When the volume wraps the allocation, loads of different waves, and in
    the strided layout the K loads of one wave, can read the same segment,
    and the repeats meet the data in a cache.  Averaged over up to
    ``max_iters`` iterations spread evenly over the run.  Assumes n_vec is a
    multiple of 64, so that every load reads one whole segment."""
    import numpy as np
    order = int(order)
    if order not in (0, 1, 2):
        raise ValueError(f"unknown order {order}")
    if Q <= 0 or n_waves <= 0 or K <= 0:
        return 0.0
    if n_vec % 64:
        raise ValueError("n_vec must be a multiple of 64")
    S = n_vec // 64
    G = -(-Q // n_waves)
    its = np.unique(np.linspace(0, G - 1, min(G, max_iters)).astype(np.int64))
    w = np.arange(n_waves, dtype=np.int64)
    j = np.arange(K, dtype=np.int64)
    total = dup = 0
    for i in its:
        q = w * G + i if order == 1 else i * n_waves + w
        q = q[q < Q]
        if q.size == 0:
            continue
        if order == 2:
            seg = (j[None, :] * Q + q[:, None]) % S
        else:
            seg = (q[:, None] * K + j[None, :]) % S
        total += seg.size
        dup += seg.size - np.unique(seg).size
    return dup / total if total else 0.0


def idle_slots(t0, t1):
    """Share of the wave slots left idle inside a launch's window:
    1 - sum of wave durations / (waves x window), from the per-wave start
    and end clock readings.  Zero when every wave runs the whole window."""
    n = len(t0)
    if n == 0:
        return 0.0
    lo, hi = min(t0), max(t1)
    win = hi - lo
    if win <= 0:
        return 0.0
    busy = sum(b - a for a, b in zip(t0, t1))
    return 1.0 - busy / (n * win)


def active_ceiling_gbps(t0, t1, in_flight_per_wave, latency_ns, peak_gbps=HBM_PEAK_GBPS):
    """Little's-law ceiling of a launch given when its waves actually ran:
    the time average, over the launch's window, of min(peak, bytes in
    flight of the waves running at that moment / latency).

    Every wave keeps at most ``in_flight_per_wave`` bytes outstanding while
    it runs and none after it ends, so the launch's rate at any moment is at
    most that minimum, and its window rate at most this average.  With
    every wave running for the whole window it is the cell's design ceiling;
    waves that finish early lower it only where the rest no longer cover
    the bandwidth-delay product."""
    n = len(t0)
    if n == 0:
        return 0.0
    ev = sorted([(a, 1) for a in t0] + [(b, -1) for b in t1])
    lo, hi = ev[0][0], max(t1)
    if hi <= lo:
        return min(peak_gbps, n * in_flight_per_wave / latency_ns)
    area, active, last = 0.0, 0, lo
    for t, d in ev:
        if t > last:
            area += (t - last) * min(peak_gbps, active * in_flight_per_wave / latency_ns)
            last = t
        active += d
    return area / (hi - lo)


def littles_ceiling_gbps(in_flight, latency_ns, peak_gbps=HBM_PEAK_GBPS):
    """Little's-law ceiling of a cell: the smaller of the datasheet figure
    and bytes in flight over the round-trip latency (bytes/ns = GB/s)."""
    if latency_ns <= 0:
        raise ValueError("latency must be positive")
    return min(peak_gbps, in_flight / latency_ns)


def gap_split(cells, peak_gbps=HBM_PEAK_GBPS):
    """Where a sweep's distance from the datasheet figure goes.

    ``cells``: dicts with the cell's issued ``bytes``, its measured
    ``gbps``, its Little's-law design ``ceiling_gbps`` (every wave running)
    and its ``active_ceiling_gbps`` (the same with the waves that actually
    ran, see :func:`active_ceiling_gbps`).  Times are summed over the cells
    (each cell's bytes at a rate), so the three factors multiply exactly:

        kernel_frac = ceiling_frac_of_peak * (1 - tail_loss) * residual_frac

    ceiling_frac_of_peak  time at the datasheet rate / time at the design
                          ceilings: what offering too few bytes in flight
                          costs by design;
    tail_loss             1 - time at the design ceilings / time at the
                          active ceilings: what the uneven finish of the
                          static equal split costs in ceiling;
    residual_frac         time at the active ceilings / measured time: how
                          far the memory system stays below what the
                          running waves offer.
    """
    if not cells:
        raise ValueError("no cells")
    t_meas = sum(c["bytes"] / c["gbps"] for c in cells)
    t_act = sum(c["bytes"] / c["active_ceiling_gbps"] for c in cells)
    t_ceil = sum(c["bytes"] / c["ceiling_gbps"] for c in cells)
    t_peak = sum(c["bytes"] / peak_gbps for c in cells)
    return {"kernel_frac": t_peak / t_meas,
            "ceiling_frac_of_peak": t_peak / t_ceil,
            "tail_loss": 1.0 - t_ceil / t_act,
            "residual_frac": t_act / t_meas,
            "frac_of_ceiling": t_ceil / t_meas}


def line_coverage(alloc_bytes, vec_bytes, issued_loads, line=128):
    """Exact 128-byte-line coverage of a cell (Section 4.2, "Allocation-size
    sweep": with no address trace the paper can only bound its unique
    coverage by issued volume over allocation).

    A cell's loads read the vector stream 0, 1, ..., issued - 1 modulo the
    allocation's vector count (every group is K consecutive 64-lane
    segments, and the groups below Q are consecutive), so after m whole
    passes and a remainder of r vectors, the lines of the first r vectors
    are read m + 1 times and all others m times.  Issued loads and the
    vector count are multiples of 64, so r covers whole lines."""
    n_vec = alloc_bytes // vec_bytes
    alloc_lines = alloc_bytes // line
    m, r = divmod(issued_loads, n_vec)
    r_lines = r * vec_bytes // line
    unique = alloc_lines if m else r_lines
    total = m * alloc_lines + r_lines
    return {"unique_lines": unique, "alloc_lines": alloc_lines, "line_reads": total,
            "re_reads": total - unique, "max_reads": m + (1 if r else 0),
            "coverage": unique / alloc_lines}


def summarize_curve(samples):
    """Summary of one response curve {K: [GB/s per launch]}."""
    med = per_k_medians(samples)
    out = {
        "median_gbps": {int(k): v for k, v in sorted(med.items())},
        "best_gbps": {int(k): max(v) for k, v in sorted(samples.items())},
        "min_gbps": {int(k): min(v) for k, v in sorted(samples.items())},
        "peak_K": peak_k(med),
        "knee_K": knee(med),
        "regime": classify(med) if len(med) >= 3 else None,
        "launches": sum(len(v) for v in samples.values()),
        "anomalous": [(int(k), x, r) for k, x, r in anomalous_launches(samples)],
    }
    if 2 in med and 8 in med:
        out["decline_2_8"] = decline(med[2], med[8])
        out["paired_declines_2_8"] = paired_declines(samples)
    return out
