"""CPU oracle of the USP-ESBGK step (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package; the product path never does.
"""
