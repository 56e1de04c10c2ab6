"""MI355X-native homomorphic convolution layers (FFConv, arXiv 2102.03494).

``he``      -- thin binding of the C ABI (include/ffconv_he.h), torch tensors
               for device memory and streams;
``client``  -- key generation, encryption and decryption (secret-key holder);
``layers``  -- server-side packing layouts, plaintext weights and scales;
``build``   -- compiles libffconv_he.so for gfx950 in-tree.

The HIP library is loaded on first use; if it is missing or does not load,
that use raises ImportError -- there is no other implementation to fall back to.
"""
