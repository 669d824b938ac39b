"""Lane-by-lane brute-force simulation for tiny inputs (oracle self-check).

Pure Python loops: for every wave, every iteration of that wave, every one
of the K loads and every lane, read the vector the address map names and
fold each of its 32-bit words into that lane's wrapping sum and XOR.  It
shares nothing with the vectorised code in ``checksums`` except the
buffer, so the two pin each other on small cases.
"""


def simulate(words, V, K, Q, n_waves, base=0, n_vec=None, blocked=False,
             strided=False):
    """Return per-lane sinks as a dict {(wave, lane): (sum32, xor32)}.

    Round robin: wave w takes groups w, w + n_waves, ...; blocked: wave w
    takes the w-th run of ceil(Q / n_waves) consecutive groups.  Load j of
    group q reads the segment after the group's previous load (q*K + j), or
    with ``strided`` the segment j*Q + q.
    """
    wpv = V // 4
    if n_vec is None:
        n_vec = len(words) // wpv - base
    lanes = {}
    for w in range(n_waves):
        for lane in range(64):
            lanes[(w, lane)] = [0, 0]
    per = (Q + n_waves - 1) // n_waves
    for w in range(n_waves):
        if blocked:
            q, step, stop = w * per, 1, min(Q, (w + 1) * per)
        else:
            q, step, stop = w, n_waves, Q
        while q < stop:                    # this wave's iterations
            for j in range(K):             # K independent loads
                seg = j * Q + q if strided else q * K + j
                for lane in range(64):
                    v = base + (seg * 64 + lane) % n_vec
                    acc = lanes[(w, lane)]
                    for t in range(wpv):
                        word = int(words[v * wpv + t])
                        acc[0] = (acc[0] + word) & 0xFFFFFFFF
                        acc[1] ^= word
            q += step
    return {k: (v[0], v[1]) for k, v in lanes.items()}


def per_wave(lanes, n_waves):
    """Fold a per-lane dict into per-wave (sum32, xor32) lists."""
    s = [0] * n_waves
    x = [0] * n_waves
    for (w, _lane), (ls, lx) in lanes.items():
        s[w] = (s[w] + ls) & 0xFFFFFFFF
        x[w] ^= lx
    return s, x
