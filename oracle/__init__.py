"""Test infrastructure: the float64 CPU oracle (see cdg2_oracle).  Only tests/,
the graft smoke check and the benchmark's cpu_baseline leg may import this."""
