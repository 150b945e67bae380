#!/bin/sh
# Builds the CPU oracle (test infrastructure) into oracle/liboracle.so.
# No floating-point contraction: the output-sensitive sampler's binomial
# variates are defined by their sequence of IEEE basic operations.
set -e
cd "$(dirname "$0")"
g++ -O2 -std=c++17 -Wall -Wextra -ffp-contract=off -shared -fPIC -o liboracle.so.tmp wrs_oracle.cpp wrs_oracle_os.cpp
mv liboracle.so.tmp liboracle.so
