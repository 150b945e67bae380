#!/bin/sh
# Builds the CPU oracle (test infrastructure) into oracle/liboracle.so, or,
# with arguments, into the file named by the first one with the compiler
# flags that follow (the benchmark's timed copy: -O3 -march=native).
# No floating-point contraction: the output-sensitive sampler's binomial
# variates are defined by their sequence of IEEE basic operations.
set -e
cd "$(dirname "$0")"
OUT=liboracle.so
FLAGS="-O3"
if [ $# -ge 1 ]; then
    OUT="$1"
    shift
    FLAGS="$*"
fi
g++ $FLAGS -std=c++17 -Wall -Wextra -ffp-contract=off -shared -fPIC -o "$OUT.tmp" wrs_oracle.cpp wrs_oracle_os.cpp
mv "$OUT.tmp" "$OUT"
