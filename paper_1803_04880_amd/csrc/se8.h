// Launch parameters of the per-8x8-block protection kernels (se8.hip).
#pragma once

#include <cstring>

#include "common.h"

namespace dwtfrag {

// FIPS 180-4 round constants and initial hash values, derived on the host
// from the square and cube roots of the first primes.
struct Sha2Tables {
  uint32_t k256[64];
  uint64_t k512[80];
  uint32_t h256[8];
  uint64_t h512[8];
};

struct Se8Geometry {
  uint64_t H, hb, wb, blocks;
  uint64_t priv_bytes, pub1_bytes, pub2_bytes;
};

struct Se8Params {
  const uint8_t *in;        // protect input (n bytes)
  uint8_t *priv, *pub1, *pub2;                        // protect outputs
  const uint8_t *priv_in, *pub1_in, *pub2_in;         // restore inputs
  uint8_t *out;             // restore output (n bytes)
  uint64_t n;
  uint64_t blocks;
  uint32_t W, wb;
  AesKey key;
  uint32_t m1[16];          // SHA-256 message template (key, nonce, padding)
  uint64_t m2_key[2], m2_nonce[2];
  Sha2Tables tab;
};

// 0 ok, -1 invalid (n == 0, width not a positive multiple of 8), -2 out of range
int se8_make_geometry(uint64_t n, uint32_t width, Se8Geometry *g);
void se8_fill_params(const Se8Geometry &g, uint64_t n, uint32_t width, const uint8_t key[16],
                     const uint8_t nonce[16], Se8Params *P);
hipError_t launch_se8(bool forward, const Se8Params &P, hipStream_t s);

}  // namespace dwtfrag
