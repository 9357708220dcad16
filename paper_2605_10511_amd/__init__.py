"""Data path fusion for MI355X: fused scan -> decode -> filter -> probe ->
aggregate query kernels behind a C ABI (include/dpf.h)."""
from .dpf import (Column, Context, Database, DpfError, Hash, Plan, Result, execute, exported_names,  # noqa: F401
                  load)
