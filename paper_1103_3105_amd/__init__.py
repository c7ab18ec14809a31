"""MI355X-native bulk transaction execution (He & Yu, GPUTx)."""
