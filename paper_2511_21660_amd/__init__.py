"""MI355X-native Relay-BP decoding (gfx950 HIP kernels behind a C ABI).

The decoder itself is ``librelaybp.so`` (built from ``csrc/`` by
``paper_2511_21660_amd.build.build()``); ``relaybp`` is a thin ctypes binding
that marshals torch device tensors and streams into the C ABI declared in
``include/relaybp.h``.  Importing this package does not load the library.
"""
