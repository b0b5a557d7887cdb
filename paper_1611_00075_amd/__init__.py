"""MI355X-native short-range molecular dynamics hot path (arXiv:1611.00075).

The compute path lives in the HIP library libmd.so (C ABI declared in
include/md.h); `paper_1611_00075_amd.md` is its thin ctypes binding and
`paper_1611_00075_amd.inputs` draws seeded synthetic inputs.  Importing the
package does not load the library; the first call into `md` does, and fails
loudly when it is missing.
"""
__all__ = ["inputs", "md"]
