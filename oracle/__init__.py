"""TEST INFRASTRUCTURE ONLY: sequential FP64 CPU reference of the robust reference
governor.  Imported only by tests/, __graft_entry__.smoke() and bench.py's
CPU-baseline leg; the GPU library never imports it."""
