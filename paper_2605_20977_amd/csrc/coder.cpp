// Host entropy coder: integer CDF tables and a byte-wise range coder.
//
// The context model outputs the mean and scale of a Gaussian per symbol
// (Sec. 3.1, Fig. 1), which drives the arithmetic coder. The coder stays on
// the CPU. Tables are integer and built once in float64 so that encoder and
// decoder agree bit for bit:
//   64 log-spaced scales 0.11 * exp(s * Delta), Delta = ln(64/0.11) / 63,
//   16 mean phases (m + 0.5)/16 - 0.5,
//   bins k = -R..R around the centre, R = clamp(ceil(8 sigma), 4, 255), plus
//   an escape bin holding both tails; 16-bit frequencies
//   max(1, floor(pmf * (65536 - n_bins))), the remainder to the largest bin.
// The range coder is the carry-propagating byte-output design (32-bit range,
// 64-bit low with a pending 0xFF run), renormalising below 2^24.
#include <cmath>
#include <cstring>
#include <mutex>

#include "pswa_internal.h"

namespace pswa {

namespace {

double ln_smin() { return std::log(kSigmaMin); }
double ln_smax() { return std::log(kSigmaMax); }
double delta() { return (ln_smax() - ln_smin()) / (kScales - 1); }

// Gaussian mass of the unit bin at distance v = |k - mu| from the mean,
// written so that it never subtracts two values close to 1.
double bin_mass(double v, double sigma) {
  const double s2 = sigma * std::sqrt(2.0);
  return 0.5 * (std::erfc((v - 0.5) / s2) - std::erfc((v + 0.5) / s2));
}

CdfTables build_tables() {
  CdfTables t;
  t.radius.resize(kTables);
  t.offset.resize(kTables + 1);
  t.cum_off.resize(kTables);
  const double total = double(1u << kPrecBits);
  const double sqrt2 = std::sqrt(2.0);
  uint32_t off = 0, coff = 0;
  for (int s = 0; s < kScales; ++s) {
    const double sig = kSigmaMin * std::exp(s * delta());
    const int R = int(std::fmin(255.0, std::fmax(4.0, std::ceil(8.0 * sig))));
    for (int m = 0; m < kPhases; ++m) {
      const int x = s * kPhases + m;
      const double f = (m + 0.5) / kPhases - 0.5;
      const int nb = 2 * R + 2;
      std::vector<double> pmf(nb);
      for (int k = -R; k <= R; ++k) pmf[k + R] = bin_mass(std::fabs(double(k) - f), sig);
      const double s2 = sig * sqrt2;
      const double below = 0.5 * std::erfc((f - (double(-R) - 0.5)) / s2);
      const double above = 0.5 * std::erfc(((double(R) + 0.5) - f) / s2);
      pmf[nb - 1] = below + above;
      std::vector<int64_t> fq(nb);
      int64_t sum = 0;
      for (int b = 0; b < nb; ++b) {
        fq[b] = std::max<int64_t>(1, int64_t(std::floor(pmf[b] * (total - nb))));
        sum += fq[b];
      }
      int big = 0;
      for (int b = 1; b < nb; ++b)
        if (fq[b] > fq[big]) big = b;
      fq[big] += int64_t(total) - sum;
      t.radius[x] = uint32_t(R);
      t.offset[x] = off;
      t.cum_off[x] = coff;
      uint32_t c = 0;
      t.cum.push_back(0);
      for (int b = 0; b < nb; ++b) {
        t.freq.push_back(uint16_t(fq[b] == 65536 ? 0 : fq[b]));
        c += uint32_t(fq[b]);
        t.cum.push_back(c);
      }
      off += nb;
      coff += nb + 1;
    }
  }
  t.offset[kTables] = off;
  return t;
}

}  // namespace

const CdfTables& cdf_tables() {
  static std::once_flag once;
  static CdfTables tables;
  std::call_once(once, [] { tables = build_tables(); });
  return tables;
}

float ln_sigma_min_f32() { return float(ln_smin()); }
float inv_delta_f32() { return float(1.0 / delta()); }

// ----------------------------------------------------------- encoder

void RangeEncoder::put(uint8_t b) {
  if (n_ < cap_)
    out_[n_] = b;
  else
    overflow_ = true;
  ++n_;
}

void RangeEncoder::shift_low() {
  if (uint32_t(low_) < 0xFF000000u || (low_ >> 32) != 0) {
    const uint8_t carry = uint8_t(low_ >> 32);
    uint8_t temp = cache_;
    do {
      put(uint8_t(temp + carry));
      temp = 0xFF;
    } while (--cache_size_ != 0);
    cache_ = uint8_t(low_ >> 24);
  }
  ++cache_size_;
  low_ = (low_ & 0x00FFFFFFu) << 8;
}

void RangeEncoder::encode(uint32_t start, uint32_t size) {
  range_ >>= kPrecBits;
  low_ += uint64_t(start) * range_;
  range_ *= size;
  while (range_ < (1u << 24)) {
    range_ <<= 8;
    shift_low();
  }
}

void RangeEncoder::bit(uint32_t b) { encode(b ? 0x8000u : 0u, 0x8000u); }

void RangeEncoder::symbol(int32_t v, int32_t center, uint16_t index) {
  const CdfTables& t = cdf_tables();
  const int R = int(t.radius[index]);
  const uint32_t* cum = &t.cum[t.cum_off[index]];
  const int64_t k = int64_t(v) - int64_t(center);
  if (k >= -R && k <= R) {
    const int b = int(k) + R;
    encode(cum[b], cum[b + 1] - cum[b]);
    return;
  }
  const int esc = 2 * R + 1;
  encode(cum[esc], cum[esc + 1] - cum[esc]);
  bit(k < 0 ? 1u : 0u);
  const uint64_t e = uint64_t(k < 0 ? -k : k) - uint64_t(R) - 1;  // >= 0
  const uint64_t n = e + 1;
  int nb = 0;
  while ((n >> (nb + 1)) != 0) ++nb;
  for (int i = 0; i < nb; ++i) bit(0);
  for (int i = nb; i >= 0; --i) bit(uint32_t((n >> i) & 1u));
}

void RangeEncoder::finish() {
  for (int i = 0; i < 5; ++i) shift_low();
}

// ----------------------------------------------------------- decoder

RangeDecoder::RangeDecoder(const uint8_t* in, size_t n) : in_(in), n_(n) {
  for (int i = 0; i < 5; ++i) code_ = (code_ << 8) | next();
}

uint32_t RangeDecoder::next() {
  if (p_ < n_) return in_[p_++];
  // A well-formed stream is fully consumed by its own renormalisations;
  // reading past its end by more than the flush length means truncation.
  if (++overrun_ > 4) ok_ = false;
  return 0;
}

bool RangeDecoder::bit(uint32_t* b) {
  range_ >>= kPrecBits;
  const uint32_t v = code_ / range_;
  *b = v >= 0x8000u ? 1u : 0u;
  code_ -= (*b ? 0x8000u : 0u) * range_;
  range_ *= 0x8000u;
  while (range_ < (1u << 24)) {
    code_ = (code_ << 8) | next();
    range_ <<= 8;
  }
  if (v >= 0x10000u) ok_ = false;
  return ok_;
}

bool RangeDecoder::symbol(int32_t center, uint16_t index, int32_t* out) {
  if (!ok_) return false;
  const CdfTables& t = cdf_tables();
  if (index >= kTables) return ok_ = false;
  const int R = int(t.radius[index]);
  const int nb = 2 * R + 2;
  const uint32_t* cum = &t.cum[t.cum_off[index]];
  range_ >>= kPrecBits;
  const uint32_t v = code_ / range_;
  if (v >= (1u << kPrecBits)) return ok_ = false;
  int lo = 0, hi = nb;  // find b with cum[b] <= v < cum[b+1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (cum[mid] <= v)
      lo = mid;
    else
      hi = mid;
  }
  const int b = lo;
  code_ -= cum[b] * range_;
  range_ *= cum[b + 1] - cum[b];
  while (range_ < (1u << 24)) {
    code_ = (code_ << 8) | next();
    range_ <<= 8;
  }
  if (b < 2 * R + 1) {
    *out = int32_t(int64_t(center) + b - R);
    return ok_;
  }
  uint32_t neg = 0;
  if (!bit(&neg)) return false;
  int zeros = 0;
  uint32_t x = 0;
  for (;;) {
    if (!bit(&x)) return false;
    if (x) break;
    if (++zeros > 40) return ok_ = false;
  }
  uint64_t n = 1;
  for (int i = 0; i < zeros; ++i) {
    if (!bit(&x)) return false;
    n = (n << 1) | x;
  }
  const int64_t mag = int64_t(n - 1) + R + 1;
  const int64_t val = int64_t(center) + (neg ? -mag : mag);
  if (val < INT32_MIN || val > INT32_MAX) return ok_ = false;
  *out = int32_t(val);
  return ok_;
}

}  // namespace pswa
