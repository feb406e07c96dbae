/*
 * lk_wire.h -- memory layout shared by the host library and the persistent worker
 * kernel.  Private to the library (the public API is include/lk.h).
 *
 * Dual mailbox (Sec. 2.4, Fig. 2): per worker, a to_GPU command ring written by the host
 * and a from_GPU status ring written by the worker, both in fine-grained host-coherent
 * memory.  Table 1 gives the codes but no transitions; every mailbox word therefore
 * carries a sequence number beside its code, word = (seq << 8) | code, which makes the
 * handshake two-phase and lets one slot be reused without a reset through NOP.
 *
 * Both directions move whole 64-byte records in one PCIe transaction:
 *   - command slot (to_GPU): the worker reads the slot with one 64-byte load and accepts
 *     it only if word 0 holds the expected (seq, code) AND every other word carries the
 *     low 16 bits of that seq in its top 16 bits.  Each word is written by one aligned
 *     8-byte host store and read by one 8-byte device load, so a slot whose eight tags
 *     all match was written entirely for this seq: the descriptor arrives with its
 *     doorbell, with no second dependent read;
 *   - status slot (from_GPU): the worker writes the whole record with one 64-byte store
 *     (one full-line posted write, no partial-line merge on the host side), tagged the
 *     same way; the host accepts it once word 0 shows the seq and all tags match.
 * Rings are padded so that every mailbox starts on its own 128-byte boundary.
 */
#ifndef LK_WIRE_H
#define LK_WIRE_H

#include <stdint.h>

/* Table 1, to_GPU values. */
#define LKW_TO_NOP 4u
#define LKW_TO_EXIT 8u
#define LKW_TO_WORK 16u /* WORK = 16 + op */

/* Table 1, from_GPU values, plus three values Table 1 leaves unused. */
#define LKW_FROM_INIT 0u
#define LKW_FROM_FINISHED 1u
#define LKW_FROM_WORKING 2u
#define LKW_FROM_ERROR 3u    /* extension: descriptor rejected */
#define LKW_FROM_NOP 4u
#define LKW_FROM_EXITED 5u   /* extension: worker left the loop on EXIT */
#define LKW_FROM_TIMEDOUT 6u /* extension: worker left the loop on its idle watchdog */

#define LKW_WORD(seq, code) (((uint64_t)(seq) << 8) | (uint64_t)(code))
#define LKW_SEQ(word) ((word) >> 8)
#define LKW_CODE(word) ((uint32_t)((word) & 0xffu))

#define LKW_TAG_SHIFT 48
#define LKW_PAYLOAD_MASK ((1ull << LKW_TAG_SHIFT) - 1)
#define LKW_TAG(seq) ((uint64_t)((seq) & 0xffffu) << LKW_TAG_SHIFT)

/* Command slot: 8 tagged words.  Words 1..7 = tag | 48-bit payload. */
enum {
  LKW_W_DOORBELL = 0, /* (seq << 8) | code, written last with release semantics */
  LKW_W_N = 1,        /* element count of this slice */
  LKW_W_IN = 2,       /* device address of the slice's input */
  LKW_W_OUT = 3,      /* device address of the slice's output */
  LKW_W_AUX = 4,      /* device address: this member's partial-result entry (AFFINE, SUM),
                         the slice's y (AXPY), the tile counter (BATCH), or 0 */
  LKW_W_A = 5,        /* uint32 a | (member index << 32) */
  LKW_W_B = 6,        /* uint32 b | (descriptor flags << 32) */
  LKW_W_ALPHA = 7,    /* float alpha bits */
  LKW_CMD_WORDS = 8
};

typedef struct lkw_cmd {
  uint64_t w[LKW_CMD_WORDS];
} lkw_cmd; /* 64 bytes */

/* Status slot: 8 tagged words written by one 64-byte device store. */
enum {
  LKW_S_WORD = 0,     /* (seq << 8) | from_GPU code */
  LKW_S_PART_LO = 1,  /* low 32 bits of this member's int64 result */
  LKW_S_PART_HI = 2,  /* high 32 bits */
  LKW_S_T_PICK = 3,   /* device wall clock at pickup (48 bits) */
  LKW_S_T_DONE = 4,   /* device wall clock before publication (48 bits) */
  LKW_S_HWID = 5,     /* HW_ID (32 bits) | XCC_ID << 32 */
  LKW_S_WORDS = 8     /* words 6..7: tag only */
};

typedef struct lkw_status {
  uint64_t w[LKW_S_WORDS];
} lkw_status; /* 64 bytes */

/* Ring stride in slots: depth rounded up to an even count (128-byte multiple). */
#define LKW_RING_STRIDE(depth) (((depth) + 1u) & ~1u)

/* Per-worker boot/liveness record, written by the worker. */
typedef struct lkw_worker {
  uint64_t word;      /* (0 << 8) | INIT at boot; (seq << 8) | EXITED / TIMEDOUT at exit */
  uint32_t hwid, xcc; /* placement read at boot */
  uint32_t wg;        /* workgroup index that claimed this mailbox */
  uint32_t pad0;
  uint64_t heartbeat; /* bumped while idle-polling */
  uint64_t t_boot;    /* device wall clock at boot */
  uint64_t t_exit;    /* device wall clock when the worker left the loop */
  uint64_t pad[10];
} lkw_worker; /* 128 bytes */

/* Device log record (device memory). */
typedef struct lkw_log {
  uint32_t seq;
  uint16_t code;
  uint16_t mailbox;
  uint32_t xcc, hwid;
  uint64_t t_pick, t_done;
} lkw_log; /* 32 bytes */

/* Kernel parameter block, passed by value. */
typedef struct lkw_params {
  lkw_cmd *cmd;          /* [n_workers][LKW_RING_STRIDE(depth)], host-coherent */
  lkw_status *status;    /* [n_workers][LKW_RING_STRIDE(depth)], host-coherent */
  lkw_worker *workers;   /* [n_workers], host-coherent */
  lkw_log *log;          /* [n_workers][log_cap], device memory, or null */
  uint32_t *claim;       /* device counter: mailbox claim at boot */
  uint32_t n_workers;
  uint32_t depth;
  uint32_t log_cap;
  uint32_t poll_sleep;
  uint32_t flags;        /* LKW_K_* */
  uint32_t threads;      /* workgroup size (the worker reads no implicit kernel argument) */
  uint64_t idle_ticks;   /* watchdog, device wall-clock ticks */
  int32_t first_delay;   /* s_sleep(1) units before the first poll after a completion; -1 = adaptive */
  uint32_t b2b_ticks;    /* a command found this soon after a completion counts as back-to-back */
  uint32_t lds_bytes;    /* dynamic LDS of each worker (the pinned-input buffer) */
  uint32_t la_ticks;     /* look-ahead only after an item that ran at least this long */
  uint32_t xcc_mask;     /* a workgroup whose XCC_ID bit is clear leaves at boot */
  uint32_t pad;
} lkw_params;

/* Descriptor flags, carried in bits 32..47 of LKW_W_B (same values as LK_DF_*). */
#define LKW_DF_PIN_INPUT 0x1u
#define LKW_DF_PIN_RELOAD 0x2u
// Pinned slices a worker keeps at once (its LDS table: address, length, LDS offset).
#define LKW_PIN_SLOTS 4u

#define LKW_K_REPORT_WORKING 0x1u
#define LKW_K_NO_ACQUIRE 0x2u
#define LKW_K_NO_LOOKAHEAD 0x4u

/* Dynamic LDS requested per worker so that two workers never fit on one CU
 * (160 KiB of LDS per CU on gfx950). */
#define LKW_LDS_PAD_BYTES (96u * 1024u)

#endif /* LK_WIRE_H */
