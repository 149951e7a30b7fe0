"""CPU oracle for round-synchronous peeling and IBLT listing.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the library itself never does.  It
shares no code with the HIP library (``paper_1302_7014_amd``) and never imports
it.  Its inputs come from ``workloads`` (seeded generators only).
"""
