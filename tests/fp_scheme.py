"""A binary32 model of the streaming sum's whole accumulation scheme, for
pinning the error bound (test helper; not the oracle).

Every lane runs Sum2 (Ogita, Rump and Oishi, 2005): TwoSum (Knuth) of the
running sum and each term, the errors summed plainly.  Pairs (s, c) are
merged by TwoSum of the s parts and a plain sum of the c parts and the
TwoSum error.  A wave merges its 64 lanes in four cross-lane steps (lane i
with lane i^1, then i^2, then the quads 4 and 8 lanes away within a row of
16) and then the four rows as a tree of two levels; a workgroup merges its
four waves as a tree of two levels; so a workgroup's pair is the root of a
tree of depth 8 over its lanes.  The workgroup pairs are widened to binary64
and combined by 256 threads: thread t adds s_i + c_i of pairs i = t, t+256,
... in turn, then the thread totals meet in a binary tree.

Which lane the rotation steps pair with changes only the pairing inside a
level, not the depth; the model rotates towards lower lanes.
"""
import numpy as np

f32 = np.float32


def two_sum(a, b):
    s = f32(a + b)
    bb = f32(s - a)
    e = f32(f32(a - f32(s - bb)) + f32(b - bb))
    return s, e


def lane_sum2(terms):
    s, c = f32(0), f32(0)
    for x in terms:
        s, e = two_sum(s, f32(x))
        c = f32(c + e)
    return s, c


def lane_plain(terms):
    s = f32(0)
    for x in terms:
        s = f32(s + f32(x))
    return s, f32(0)


def merge(a, b):
    s, e = two_sum(a[0], b[0])
    return s, f32(f32(a[1] + b[1]) + e)


def merge_plain(a, b):
    return f32(a[0] + b[0]), f32(0)


def _src(step, i):
    if step == 0:
        return i ^ 1
    if step == 1:
        return i ^ 2
    n = 4 if step == 2 else 8
    return (i & ~15) | ((i - n) & 15)


def wave(pairs, mg=merge):
    p = list(pairs)
    assert len(p) == 64
    for step in range(4):
        p = [mg(p[i], p[_src(step, i)]) for i in range(64)]
    r = [p[0], p[16], p[32], p[48]]
    return mg(mg(r[0], r[1]), mg(r[2], r[3]))


def workgroup(waves, mg=merge):
    assert len(waves) == 4
    return mg(mg(waves[0], waves[1]), mg(waves[2], waves[3]))


def final_combine(partials, threads=256):
    acc = [0.0] * threads
    for i, (s, c) in enumerate(partials):
        acc[i % threads] = acc[i % threads] + (float(s) + float(c))
    h = threads // 2
    while h:
        for t in range(h):
            acc[t] = acc[t] + acc[t + h]
        h //= 2
    return acc[0]


def scheme(lane_terms, compensated=True):
    """Sum of ``lane_terms`` (a list over workgroups of 256 lists of terms,
    lanes in wave order) through the whole scheme; ``compensated=False``
    gives the same layout with plain binary32 sums instead."""
    lane = lane_sum2 if compensated else lane_plain
    mg = merge if compensated else merge_plain
    partials = []
    for wg in lane_terms:
        assert len(wg) == 256
        pairs = [lane(t) for t in wg]
        ws = [wave(pairs[64 * k: 64 * k + 64], mg) for k in range(4)]
        partials.append(workgroup(ws, mg))
    return final_combine(partials)
