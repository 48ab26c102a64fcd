"""MI355X-native Sorted Opacity Fields hot path: HIP kernels behind a C ABI (libsof.so)
and a thin ctypes binding.  Importing the package does not load the library; the first
call into `paper_2506_19139_amd.sof` does, and fails loudly if it is not built."""

__all__ = ["sof", "scenes"]
