"""MI355X-native SZ dual-quantisation (vecSZ hot path, arXiv 2201.04614).

Compress: prequantisation q = round(x / (2 eb)), blockwise 1/2/3-D Lorenzo
prediction on q with zero / block-mean / edge-mean / global-mean padding,
uint16 codes within a radius, block-major outlier list. Decompress: the exact
inverse (outlier scatter, blockwise prefix sum, dequantisation). All of it runs
in the hand-written HIP kernels of libdq.so (include/dq.h); this package is
the Python binding.
"""

from .binding import (DQ_ECAPACITY, DQ_ECORRUPT, DQ_EDEVICE, DQ_EINVAL, DQ_ENOTSUP,  # noqa: F401
                      DQ_ERANGE, DQ_OK, Codec, DQError, DQStream, Hook, compress,
                      decompress, lib, make_params, pad_count, validate)
