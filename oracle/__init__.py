"""CPU oracle for the offered-ILP streaming-load path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
calls anything in this directory; only the test-suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may use it.

The oracle is a plain, slow, obviously-correct restatement of what the paper's
method computes (Manjunath & Ramachandra, "Concurrency Response of Plain
Global Loads on the NVIDIA H100"):

* ``splitmix``  - the seeded counter-based buffer generator (SplitMix64 of
  Steele, Lea and Flood, 2014), written from its published definition.
* ``plan``      - the fixed-work control of Section 3 ("Fixed-work control")
  and the exact-work accounting of Section 4.2 ("Exact-work accounting"):
  iteration counts, issued logical loads and the K-set mismatch.
* ``checksums`` - the address map (Section 3: whatever K is, a wave's
  loads stay one contiguous, coalesced run; K only sets how many loads
  each lane has outstanding) and the per-lane / per-wave / global wrapping-sum and XOR
  sinks of Section 3 ("Instruments").
* ``brute``     - a lane-by-lane pure-Python simulation for tiny inputs, used
  to pin ``checksums``.
* ``fpsum``     - exact sums of FP32 / BF16 / FP8-e4m3 payloads and the
  compensated-summation error bound used by the precision variant.

Every integer result has exactly one correct value; floating-point sums are
exact (rounded once to FP64 at the end).
"""
