// Compiled tile shapes (BLOCK threads x IPT items per thread).  The selection
// kernel carries the full sweep of section 3.3 (IPT 1, 2, 4 and beyond); the
// other kernels use vector-width IPTs only.
#pragma once

#define CRYSTAL_VARIANTS_ALL(X)                                                  \
    X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(64, 16)                                \
    X(128, 1) X(128, 2) X(128, 4) X(128, 8) X(128, 16)                           \
    X(256, 1) X(256, 2) X(256, 4) X(256, 8) X(256, 16)                           \
    X(512, 1) X(512, 2) X(512, 4) X(512, 8) X(512, 16)                           \
    X(1024, 1) X(1024, 2) X(1024, 4) X(1024, 8) X(1024, 16)

#define CRYSTAL_VARIANTS_VEC(X)                                                  \
    X(64, 4) X(64, 8) X(64, 16)                                                  \
    X(128, 4) X(128, 8) X(128, 16)                                               \
    X(256, 4) X(256, 8) X(256, 16)                                               \
    X(512, 4) X(512, 8) X(512, 16)                                               \
    X(1024, 4) X(1024, 8) X(1024, 16)

// Radix partitioning: one thread per digit, so at least 256 threads.
#define CRYSTAL_VARIANTS_RADIX(X)                                                \
    X(256, 4) X(256, 8) X(256, 16)                                               \
    X(512, 4) X(512, 8) X(512, 16)                                               \
    X(1024, 4) X(1024, 8) X(1024, 16)

#define CRYSTAL_VARIANT_KEY(B, I) ((B) * 1000 + (I))
