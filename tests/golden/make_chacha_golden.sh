#!/bin/sh
# Writes chacha20_openssl.txt: ChaCha20 keystream (RFC 8439 block function) from
# the openssl CLI, used to pin the oracle's block function.  openssl's -iv is the
# 32-bit little-endian block counter followed by the 96-bit nonce.
set -e
cd "$(dirname "$0")"
out=chacha20_openssl.txt
: > $out
for spec in \
  "000102030405060708090a0b0c0d0e0f101112131415161718191a1b1c1d1e1f 01000000 000000090000004a00000000" \
  "0700000000000000010000000000000002000000000000004845514701000000 00000000 030000000000000000000000" \
  "ffffffffffffffff040000000000000033221100000000004845514701000000 05000000 000000000000000000000000"
do
  set -- $spec
  key=$1; ctr=$2; nonce=$3
  ks=$(head -c 128 /dev/zero | openssl enc -chacha20 -K "$key" -iv "$ctr$nonce" | od -An -tx1 -v | tr -d ' \n')
  echo "$key $ctr $nonce $ks" >> $out
done
