"""Adaptive image ray-tracing (Parkin 2010) on MI355X.

`inputs` holds the seeded synthetic workloads; `air` is the binding to the
HIP library libair.so (include/air.h).  Importing the package loads nothing;
the library is loaded on first use and there is no CPU fallback."""
