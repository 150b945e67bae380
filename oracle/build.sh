#!/bin/sh
# Builds the CPU oracle (test infrastructure) into oracle/liboracle.so.
set -e
cd "$(dirname "$0")"
g++ -O2 -std=c++17 -Wall -Wextra -shared -fPIC -o liboracle.so.tmp wrs_oracle.cpp
mv liboracle.so.tmp liboracle.so
