// Shape of the cost-model network (12 -> 64 -> 64 -> 1, ReLU, float32) and
// the order of its flat parameter vector: W1 (64 x 12, row-major, output by
// input), b1 (64), W2 (64 x 64, row-major), b2 (64), w3 (64), b3 (1).
#pragma once

namespace race {

constexpr int kMlpIn = 12;
constexpr int kMlpHid = 64;
constexpr int kMlpParams = kMlpHid * kMlpIn + kMlpHid + kMlpHid * kMlpHid + kMlpHid + kMlpHid + 1;

}  // namespace race
