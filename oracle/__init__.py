"""CPU oracle of the PHIA sweep -- test infrastructure only.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The device library never does.
"""
